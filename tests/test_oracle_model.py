"""Pins of the oracle network, forces and virial (CPU only).

The paper prints no model outputs, so the oracle is pinned by what the method
and the mathematics fix: the loop-form evaluation of the paper's equations on
tiny inputs; central finite differences of the energy; E(3) invariance with
covariant forces (full O(3), section "Training details"); same-species
permutation invariance; zero net force; virial against strained energies;
strict locality (section "Allegro: Scalable Equivariant Deep Learning"); a
ghost-shell box reproducing the periodic box; the pair-potential limit when
every path weight is zero; continuity at the cutoff; NVE energy conservation.
Per-ordered-species-pair cutoffs (section "Species-dependent cutoffs") get the
loop form, finite differences and continuity at each pair's own cutoff.  The
ZBL repulsion (section "Training details") is pinned by its Coulomb limit
(the screening function is 1 at zero separation), the dimer with a silent
network, finite differences, continuity at the cutoff and its symmetry; its
published constants themselves have no printed value to compare with here.
"""
import copy
import math

import numpy as np
import pytest

import workloads as W
from oracle import md, model
from oracle.neighbors import neighbor_list

import oracle_loops


def tiny_model(l_max=2, n_layers=2, n=4, d=8, S=2, rc=3.0, mix=True):
    return W.ModelConfig(n_species=S, r_cut=rc, l_max=l_max, n_layers=n_layers, n_tensor=n,
                         twobody_dims=(d, d), latent_dims=(d, d), edge_dims=(6,), channel_mix=mix)


def cluster(n_atoms, seed, S=2):
    rng = np.random.default_rng(seed)
    pos = W.random_packed_cluster(n_atoms, rng, 0.9)
    sp = W.assign_species(n_atoms, [1] * S, rng)
    return W.System(pos=pos, species=sp, cell=np.zeros(3), pbc=np.zeros(3, np.int32), n_local=n_atoms)


def weights(mc, seed):
    return W.make_weights(mc, np.random.default_rng(seed))


def rot(seed, reflect=False):
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q *= np.sign(np.diag(r))
    if (np.linalg.det(q) < 0) != reflect:
        q[:, 0] *= -1
    return q


@pytest.mark.parametrize("l_max,n_layers,mix", [(2, 2, True), (1, 1, True), (2, 2, False), (1, 2, True)])
def test_matches_loop_form(l_max, n_layers, mix):
    mc = tiny_model(l_max, n_layers, mix=mix)
    w = weights(mc, 11)
    s = cluster(9, 3)
    ref = oracle_loops.energy(mc, w, s)
    got = model.evaluate(mc, w, s).edge_energy
    assert ref.shape == got.shape and len(ref) > 20
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("l_max,n_layers,n_atoms", [(2, 3, 8), (1, 4, 8), (3, 3, 6), (3, 2, 7)])
def test_deep_matches_loop_form(l_max, n_layers, n_atoms):
    """Three or more layers bring unnatural-parity irreps (parity blocks of the
    strided layout, the triple-product couplings, per-irrep mixing); l_max 3
    brings the l = 3 harmonics."""
    mc = tiny_model(l_max, n_layers, n=3, d=8)
    w = weights(mc, 21 + n_layers)
    s = cluster(n_atoms, 4)
    ref = oracle_loops.energy(mc, w, s)
    got = model.evaluate(mc, w, s).edge_energy
    assert ref.shape == got.shape and len(ref) > 10
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-13)


def test_periodic_loop_form():
    mc = tiny_model(2, 2)
    w = weights(mc, 2)
    s = W.jittered_lattice_box(8, 4.3, 0.3, W.WATER_MIX, 9, sites_per_side=2)  # box < 2 r_c: many images
    ref = oracle_loops.energy(mc, w, s)
    got = model.evaluate(mc, w, s).edge_energy
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-13)


def _fd_check(mc, w, s, comps, h=1e-5, tol=2e-7, scale=None, shift=None):
    r = model.evaluate(mc, w, s, scale, shift)
    p = model.Params(mc, w)
    for (a, ax) in comps:
        xp, xm = s.pos.copy(), s.pos.copy()
        xp[a, ax] += h
        xm[a, ax] -= h
        ep = model.energy_of_positions(mc, w, s, xp, scale, shift, params=p)
        em = model.energy_of_positions(mc, w, s, xm, scale, shift, params=p)
        fd = -(ep - em) / (2 * h)
        assert abs(fd - r.forces[a, ax]) < tol, (a, ax, fd, r.forces[a, ax])


def test_forces_finite_difference_periodic():
    mc, s, w = W.workload(1)
    rng = np.random.default_rng(0)
    comps = [(int(rng.integers(64)), int(rng.integers(3))) for _ in range(6)]
    sc, sh = W.species_scale_shift(mc, np.random.default_rng(1))
    _fd_check(mc, w, s, comps, scale=sc, shift=sh)


def test_forces_finite_difference_two_layers():
    mc = tiny_model(2, 2, n=6, d=16, rc=3.2)
    w = weights(mc, 4)
    s = cluster(14, 5)
    _fd_check(mc, w, s, [(a, ax) for a in (0, 5, 13) for ax in range(3)])


def test_forces_finite_difference_deep():
    mc = tiny_model(3, 3, n=4, d=16, rc=3.2)
    w = weights(mc, 14)
    s = cluster(12, 15)
    _fd_check(mc, w, s, [(a, ax) for a in (0, 7, 11) for ax in range(3)])


@pytest.mark.parametrize("l_max,n_layers", [(2, 2), (2, 3), (3, 3), (1, 4)])
def test_invariances_and_covariant_forces(l_max, n_layers):
    """E(3) with reflections: a path whose output parity were mislabelled would
    leave a pseudoscalar in the energy and break the mirror case."""
    mc = tiny_model(l_max, n_layers, n=6, d=16, rc=3.2)
    w = weights(mc, 6)
    s = cluster(20, 7)
    r0 = model.evaluate(mc, w, s)
    for k, refl in ((1, False), (2, True)):
        R = rot(k, refl)
        s2 = copy.copy(s)
        s2.pos = s.pos @ R.T + np.array([3.1, -2.0, 0.7])
        r1 = model.evaluate(mc, w, s2)
        assert abs(r1.energy - r0.energy) < 1e-11 * max(1, abs(r0.energy))
        assert np.allclose(r1.atom_energy, r0.atom_energy, atol=1e-11)
        assert np.allclose(r1.forces, r0.forces @ R.T, atol=1e-11)
    # permutation of two same-species atoms (and of the atom order in general)
    perm = np.random.default_rng(8).permutation(s.n_local)
    s3 = copy.copy(s)
    s3.pos, s3.species = s.pos[perm], s.species[perm]
    r3 = model.evaluate(mc, w, s3)
    assert abs(r3.energy - r0.energy) < 1e-11
    assert np.allclose(r3.forces, r0.forces[perm], atol=1e-11)


def test_periodic_box_cubic_symmetry_and_net_force():
    mc, s, w = W.workload(1)
    r0 = model.evaluate(mc, w, s)
    assert np.abs(r0.forces.sum(0)).max() < 1e-12
    s2 = copy.copy(s)
    s2.pos = s.pos[:, [1, 2, 0]]            # proper rotation mapping the cube onto itself
    r1 = model.evaluate(mc, w, s2)
    assert abs(r1.energy - r0.energy) < 1e-11
    s3 = copy.copy(s)
    s3.pos = np.mod(s.pos + np.array([1.3, -4.2, 2.2]), s.cell)
    assert abs(model.evaluate(mc, w, s3).energy - r0.energy) < 1e-11


def test_virial():
    # cluster: W = sum_i x_i (x) F_i exactly
    mc = tiny_model(2, 2, n=6, d=16, rc=3.2)
    w = weights(mc, 9)
    s = cluster(16, 10)
    r = model.evaluate(mc, w, s)
    assert np.allclose(r.virial, np.einsum("ia,ib->ab", s.pos, r.forces), atol=1e-11)
    assert np.allclose(r.atom_virial.sum(0), r.virial, atol=1e-12)
    # periodic box: W_aa = -dE/d(eps_aa) under a uniaxial strain
    mc, s, w = W.workload(1)
    r = model.evaluate(mc, w, s)
    p = model.Params(mc, w)
    h = 1e-6
    for ax in range(3):
        es = []
        for sg in (1, -1):
            s2 = copy.copy(s)
            f = np.ones(3)
            f[ax] += sg * h
            s2.pos, s2.cell = s.pos * f, s.cell * f
            es.append(model.evaluate(mc, w, s2, params=p, need_atom_virial=False).energy)
        assert abs(-(es[0] - es[1]) / (2 * h) - r.virial[ax, ax]) < 1e-6


def test_locality():
    mc = tiny_model(2, 2, n=6, d=16, rc=3.0)
    w = weights(mc, 12)
    s = cluster(30, 13)
    r0 = model.evaluate(mc, w, s)
    i0 = 0
    dist = np.linalg.norm(s.pos - s.pos[i0], axis=1)
    far = int(np.argmax(dist))
    near = int(np.argsort(dist)[1])
    assert dist[far] > mc.r_cut + 0.5
    s2 = copy.copy(s)
    s2.pos = s.pos.copy()
    # move the far atom around, keeping it outside the cutoff sphere of atom 0
    s2.pos[far] += 0.3 * (s.pos[far] - s.pos[i0]) / dist[far]
    r1 = model.evaluate(mc, w, s2)
    assert r1.atom_energy[i0] == r0.atom_energy[i0]
    s2.pos = s.pos.copy()
    s2.pos[near] += np.array([0.05, -0.03, 0.02])
    assert abs(model.evaluate(mc, w, s2).atom_energy[i0] - r0.atom_energy[i0]) > 1e-8


def test_ghost_shell_equals_periodic():
    mc, s, w = W.workload(1)
    r0 = model.evaluate(mc, w, s)
    g = W.ghost_shell(s, mc.r_cut + 1.0)
    r1 = model.evaluate(mc, w, g)
    assert np.allclose(r1.atom_energy, r0.atom_energy, atol=1e-12)
    F = r1.forces[:s.n_local].copy()
    np.add.at(F, g.ghost_owner, r1.forces[s.n_local:])
    assert np.allclose(F, r0.forces, atol=1e-12)


def test_domain_decomposition_emulated():
    """Split the periodic box into 8 subdomains, each with its own ghost shell
    (one GPU's share each); subdomain atom energies and folded forces equal the
    whole-box result."""
    mc, s, w = W.workload(1)
    r0 = model.evaluate(mc, w, s)
    half = s.cell / 2
    E = np.zeros(s.n_local)
    F = np.zeros((s.n_local, 3))
    for cx in range(2):
        for cy in range(2):
            for cz in range(2):
                c = np.array([cx, cy, cz])
                lo, hi = c * half, (c + 1) * half
                own = np.nonzero(np.all((s.pos >= lo) & (s.pos < hi), axis=1))[0]
                pos_l, idx_g = [], []
                for sx in (-1, 0, 1):
                    for sy in (-1, 0, 1):
                        for sz in (-1, 0, 1):
                            p = s.pos + np.array([sx, sy, sz]) * s.cell
                            m = np.all((p > lo - mc.r_cut - 0.1) & (p < hi + mc.r_cut + 0.1), axis=1)
                            m[own] &= not (sx == 0 and sy == 0 and sz == 0)
                            pos_l.append(p[m]); idx_g.append(np.nonzero(m)[0])
                gpos, gidx = np.concatenate(pos_l), np.concatenate(idx_g)
                sub = W.System(pos=np.concatenate([s.pos[own], gpos]),
                               species=np.concatenate([s.species[own], s.species[gidx]]),
                               cell=s.cell, pbc=np.zeros(3, np.int32), n_local=len(own))
                r = model.evaluate(mc, w, sub)
                E[own] = r.atom_energy
                np.add.at(F, np.concatenate([own, gidx]), r.forces)
    assert np.allclose(E, r0.atom_energy, atol=1e-12)
    assert np.allclose(F, r0.forces, atol=1e-12)


def test_zero_paths_is_pair_potential():
    """With every path weight zero the tensor track is silent and E_ij depends
    only on (d, Z_i, Z_j): two edges with equal (d, Z_i, Z_j) in different
    environments carry equal energies."""
    mc = tiny_model(2, 2, n=4, d=8, rc=3.0)
    w = weights(mc, 14)
    for L in (1, 2):
        w[f"layer{L}.alpha"][:] = 0.0
    pos = np.array([[0.0, 0.0, 0.0], [1.7, 0.0, 0.0], [0.3, 1.1, 0.4],
                    [10.0, 0.0, 0.0], [10.0, 1.7, 0.0], [9.1, -0.8, 0.9], [11.0, 0.5, -0.9]])
    sp = np.array([0, 1, 0, 0, 1, 1, 0], dtype=np.int32)
    s = W.System(pos=pos, species=sp, cell=np.zeros(3), pbc=np.zeros(3, np.int32), n_local=7)
    r = model.evaluate(mc, w, s)
    i, j, _ = r.nbr
    e01 = r.edge_energy[(i == 0) & (j == 1)][0]
    e34 = r.edge_energy[(i == 3) & (j == 4)][0]
    assert abs(e01 - e34) < 1e-14 and abs(e01) > 1e-6
    w2 = weights(mc, 14)
    r2 = model.evaluate(mc, w2, s)
    assert abs(r2.edge_energy[(i == 0) & (j == 1)][0] - r2.edge_energy[(i == 3) & (j == 4)][0]) > 1e-8


def test_continuity_at_cutoff():
    mc = tiny_model(2, 2, n=4, d=8, rc=3.0)
    w = weights(mc, 15)
    base = np.array([[0.0, 0.0, 0.0], [1.2, 0.4, 0.0], [0.5, -1.0, 0.3]])
    sp = np.array([0, 1, 1], dtype=np.int32)
    def E(xd):
        pos = np.concatenate([base, [[-xd, 0.0, 0.0]]])   # only pair (0, 3) nears r_c
        s = W.System(pos=pos, species=np.concatenate([sp, [0]]).astype(np.int32), cell=np.zeros(3),
                     pbc=np.zeros(3, np.int32), n_local=4)
        return model.evaluate(mc, w, s).energy
    e_out = E(3.6)  # outside every cutoff sphere
    for eps in (1e-2, 1e-3):
        assert abs(E(3.0 - eps) - e_out) < 50 * eps ** 3
    assert abs(E(2.0) - e_out) > 1e-6


def test_nve_energy_conservation_scales_dt2():
    mc, s, w = W.workload(1)
    p = model.Params(mc, w)
    v0 = W.maxwell_boltzmann(s.masses, 300.0, W.seeds(1)[4])
    def ff(x):
        s2 = copy.copy(s)
        s2.pos = x
        r = model.evaluate(mc, w, s2, params=p, need_atom_virial=False)
        return r.energy, r.forces
    T = 10.0
    fl = []
    for dt in (0.5, 0.25):
        _, _, et = md.velocity_verlet(ff, s.pos, v0, s.masses, dt, int(round(T / dt)), wrap_cell=s.cell)
        fl.append(np.max(np.abs(et - et[0])))
    ratio = fl[0] / fl[1]
    assert 3.0 < ratio < 5.0, (fl, ratio)
    assert fl[1] < 1e-3


PAIR_TABLE = ((2.2, 1.3), (2.6, 3.0))   # ordered [Z_centre][Z_neighbour], r_cut 3.0


def pair_model():
    mc = tiny_model(2, 2, n=4, d=8, rc=3.0)
    mc.pair_cutoffs = PAIR_TABLE
    return mc


def test_pair_cutoffs_loop_form():
    mc = pair_model()
    w = weights(mc, 31)
    s = cluster(10, 7)
    ref = oracle_loops.energy(mc, w, s)
    got = model.evaluate(mc, w, s).edge_energy
    assert ref.shape == got.shape and len(ref) > 10
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-13)
    # fewer edges than with the single cutoff, and a different energy
    full = model.evaluate(tiny_model(2, 2, n=4, d=8, rc=3.0), w, s)
    assert len(full.edge_energy) > len(got)


def test_pair_cutoffs_forces_finite_difference():
    mc = pair_model()
    w = weights(mc, 32)
    s = cluster(14, 9)
    _fd_check(mc, w, s, [(a, ax) for a in (1, 6, 12) for ax in range(3)])


def test_continuity_at_pair_cutoff():
    """Moving a species-1 neighbour of a species-0 centre across that ordered
    pair's cutoff (1.3 A) changes the energy by O(h^3): every contribution of
    the edge carries the envelope u, which vanishes there with its first two
    derivatives; the reverse edge (cutoff 2.6 A) stays in the list."""
    mc = pair_model()
    w = weights(mc, 33)
    base = np.array([[0.0, 0.0, 0.0], [1.9, 0.6, 0.0], [0.4, -1.8, 0.5]])
    sp = np.array([0, 0, 1], dtype=np.int32)

    def E(xd, table):
        m = copy.copy(mc)
        m.pair_cutoffs = table
        pos = np.concatenate([base, [[-xd, 0.0, 0.0]]])
        s = W.System(pos=pos, species=np.concatenate([sp, [1]]).astype(np.int32), cell=np.zeros(3),
                     pbc=np.zeros(3, np.int32), n_local=4)
        return model.evaluate(m, w, s).energy

    without = ((2.2, 1.0), (2.6, 3.0))    # the same system with the 0 -> 1 pair below 1.0 A
    diffs = [E(1.3 - h, PAIR_TABLE) - E(1.3 - h, without) for h in (2e-2, 4e-3)]
    assert abs(diffs[1]) < 50 * 4e-3 ** 3
    assert abs(diffs[0] / diffs[1]) > 60       # cubic: (2e-2 / 4e-3)^3 = 125
    assert abs(E(1.0, PAIR_TABLE) - E(1.0, without)) > 1e-6


def zbl_model(S=2, pairs=False):
    mc = tiny_model(2, 2, n=4, d=8, S=S, rc=3.0)
    mc.atomic_numbers = (1, 8) if S == 2 else (1, 6, 7, 8)
    if pairs:
        mc.pair_cutoffs = PAIR_TABLE
    return mc


def test_zbl_coulomb_limit_and_repulsion():
    import torch
    from oracle import basis
    d = torch.tensor([1e-5, 1e-4, 0.3, 0.6, 1.2, 2.4], dtype=torch.float64)
    for zi, zj in ((1.0, 1.0), (1.0, 8.0), (8.0, 8.0), (6.0, 7.0)):
        e = basis.zbl_energy(d, torch.tensor(zi, dtype=torch.float64), torch.tensor(zj, dtype=torch.float64))
        coul = 14.399645 * zi * zj / d
        assert abs(float(e[0] / coul[0]) - 1.0) < 1e-3          # screening -> 1 as r -> 0
        assert torch.all(e > 0) and torch.all(e[1:] < e[:-1])   # repulsive, decreasing
        assert torch.all(e <= coul)                             # screened below bare Coulomb
        e2 = basis.zbl_energy(d, torch.tensor(zj, dtype=torch.float64), torch.tensor(zi, dtype=torch.float64))
        assert torch.allclose(e, e2, rtol=1e-15, atol=0)


def test_zbl_dimer_with_silent_network():
    """With all network weights zero only the ZBL term remains: the dimer's
    energy is the pair energy times the envelope (two ordered halves), and
    the force is minus its radial derivative (central difference)."""
    import torch
    from oracle import basis
    mc = zbl_model()
    w = {k: np.zeros_like(v) for k, v in weights(mc, 40).items()}
    for dd in (0.7, 1.6, 2.5):
        pos = np.array([[0.1, 0.2, 0.3], [0.1 + dd, 0.2, 0.3]])
        s = W.System(pos=pos, species=np.array([0, 1], np.int32), cell=np.zeros(3), pbc=np.zeros(3, np.int32),
                     n_local=2)
        r = model.evaluate(mc, w, s)
        u = basis.envelope(torch.tensor([dd / 3.0], dtype=torch.float64), 6)
        ez = basis.zbl_energy(torch.tensor([dd], dtype=torch.float64), torch.tensor(1.0, dtype=torch.float64),
                              torch.tensor(8.0, dtype=torch.float64))
        assert abs(r.energy - float(ez * u)) < 1e-12 * max(1.0, abs(r.energy))
        h = 1e-6
        ep = model.energy_of_positions(mc, w, s, pos + np.array([[0, 0, 0], [h, 0, 0]]))
        em = model.energy_of_positions(mc, w, s, pos - np.array([[0, 0, 0], [h, 0, 0]]))
        assert abs(-(ep - em) / (2 * h) - r.forces[1, 0]) < 1e-6 * max(1.0, abs(r.forces[1, 0]))
        assert abs(r.forces[0, 0] + r.forces[1, 0]) < 1e-9 * max(1.0, abs(r.forces[1, 0]))


def test_zbl_forces_finite_difference():
    mc = zbl_model(pairs=True)
    w = weights(mc, 41)
    s = cluster(12, 13)
    _fd_check(mc, w, s, [(a, ax) for a in (0, 4, 11) for ax in range(3)], tol=1e-6)


def test_zbl_continuity_at_cutoff():
    mc = zbl_model()
    w = weights(mc, 42)
    base = np.array([[0.0, 0.0, 0.0], [1.2, 0.4, 0.0], [0.5, -1.0, 0.3]])
    sp = np.array([0, 1, 1], dtype=np.int32)

    def E(xd):
        pos = np.concatenate([base, [[-xd, 0.0, 0.0]]])
        s = W.System(pos=pos, species=np.concatenate([sp, [1]]).astype(np.int32), cell=np.zeros(3),
                     pbc=np.zeros(3, np.int32), n_local=4)
        return model.evaluate(mc, w, s).energy
    e_out = E(3.6)
    for eps in (1e-2, 1e-3):
        assert abs(E(3.0 - eps) - e_out) < 50 * eps ** 3


@pytest.mark.parametrize("l_max,n_layers", [(2, 2), (3, 3)])
def test_evaluate_centres_equals_whole_system(l_max, n_layers):
    """The sampled reference of the large-box GPU tests: a subset of centres
    evaluated from their own edges gives exactly the whole evaluation's
    (unscaled) atom energies and edge gradients for those centres."""
    mc = tiny_model(l_max, n_layers, n=4, d=8, rc=3.2)
    w = weights(mc, 41)
    s = cluster(16, 42)
    whole = model.evaluate(mc, w, s)
    i, j, sh = whole.nbr
    cents = np.array([1, 5, 11, 14])
    e_raw, g = model.evaluate_centres(mc, w, s, cents, whole.nbr)
    atom_raw = np.zeros(s.n_local)
    np.add.at(atom_raw, i, whole.edge_energy)
    assert np.allclose(e_raw, atom_raw[cents], rtol=1e-12, atol=1e-13)
    for e, ge in g.items():
        assert i[e] in cents
        assert np.allclose(ge, whole.edge_grad[e], rtol=1e-10, atol=1e-13)
    assert len(g) == int(np.isin(i, cents).sum())
