"""Step-0 parity on one GPU's spatial-decomposition share at its real shape
(section "Optimized LAMMPS-Kokkos implementation": each GPU evaluates its own
atoms from a shell of ghost atoms within r_c): 1,000,000 local atoms of the
protein-like mix in a 215 A cube plus the 6 A periodic-image ghost shell
(about 1.19M atoms in all), the r_c 4 A model with 32 channels and [128, 128]
latents, evaluated in 8M-edge chunks (about 32M edges, four chunks).

The oracle evaluates sampled centres (their atom energies) and sampled atoms
(their forces) from neighbour rows of those centres only, found with a k-d
tree over all atoms and decided by the list's exact test; the GPU's rows of
the same centres must equal them bit for bit.  Tolerances as in the other
parity tests:
  FP32         |mean dE_i| <= 1e-6 eV, max |dE_i| <= 1e-5 eV, max |dF| <= 1e-4 eV/A
  BF16-mixed   |mean dE_i| <= 1e-3 eV, RMS(dF) <= 1% of RMS(F_ref)
"""
import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

import paper_2304_10061_amd as P
import workloads as W
from oracle import model as OM
from oracle.neighbors import centre_neighbors

from gpu_helpers import to_dev
from test_gpu_parity import _report

pytestmark = pytest.mark.gpu

FP32, BF16M = P.PREC_FP32, P.PREC_BF16_MIXED
N_CENTRES, N_FORCE_ATOMS = 32, 8


@pytest.fixture(scope="module")
def share():
    mc = W.model_config(4)
    w = W.make_weights(mc, W.seeds(4)[3])
    base = W.jittered_lattice_box(1_000_000, 215.0, 0.5, W.PROTEIN_MIX, 4, sites_per_side=100)
    g = W.ghost_shell(base, 6.0)
    rng = np.random.default_rng(404)
    # half the sampled centres within 6 A of a face (ghost neighbours), half anywhere
    near = np.nonzero(np.any((base.pos < 6.0) | (base.pos > 215.0 - 6.0), axis=1))[0]
    cents = np.unique(np.concatenate([rng.choice(near, N_CENTRES // 2, replace=False),
                                      rng.choice(base.n_local, N_CENTRES // 2, replace=False)]))
    atoms = cents[::max(1, len(cents) // N_FORCE_ATOMS)][:N_FORCE_ATOMS]
    # centres that have a force atom as a neighbour: local atoms within r_c
    tree = cKDTree(g.pos[:g.n_local])
    near_atoms = np.unique(np.concatenate([np.asarray(c, dtype=np.int64)
                                           for c in tree.query_ball_point(g.pos[atoms], mc.r_cut * 1.001)]))
    need = np.union1d(atoms, near_atoms)
    nbr = centre_neighbors(g.pos, mc.r_cut, np.union1d(cents, need))
    p = OM.Params(mc, w)
    e_raw, _ = OM.evaluate_centres(mc, w, g, cents, nbr, params=p)
    _, grads = OM.evaluate_centres(mc, w, g, need, nbr, params=p)
    i, j, _ = nbr
    F = np.zeros((len(atoms), 3))
    for k, a in enumerate(atoms):
        for e in np.nonzero(i == a)[0]:
            F[k] += grads[int(e)]
        for e in np.nonzero(j == a)[0]:
            F[k] -= grads[int(e)]
    return mc, w, base, g, cents, e_raw, atoms, F, nbr


@pytest.mark.parametrize("prec", [FP32, BF16M], ids=["fp32", "bf16_mixed"])
def test_subdomain_share_step0_sampled(share, prec):
    mc, w, base, g, cents, e_ref, atoms, F_ref, nbr = share
    m = P.Model(P.config_from(mc, precision=prec, edge_chunk=8_000_000), W.pack_weights(mc, w))
    m.set_ghosts(base.n_local, g.ghost_owner, g.pos[base.n_local:] - base.pos[g.ghost_owner])
    pos, sp = to_dev(g)
    out = m.evaluate(pos, sp, g.cell, g.pbc, g.n_local)
    torch.cuda.synchronize()
    assert m.num_edges() > 3 * 8_000_000          # several chunks
    # the sampled centres' neighbour rows, bit for bit
    ci, nj, sh = (t.cpu().numpy() for t in m.copy_edges())
    lo, hi = np.searchsorted(ci, cents, side="left"), np.searchsorted(ci, cents, side="right")
    got_rows = np.concatenate([nj[a:b] for a, b in zip(lo, hi)])
    i, j, _ = nbr
    want_rows = np.concatenate([j[i == c] for c in cents])
    assert np.array_equal(np.sort(got_rows), np.sort(want_rows))
    assert np.array_equal(got_rows, want_rows)     # the same (sorted) order within each row
    assert np.all(sh == 0)
    Ea = out["atom_energy"].cpu().numpy()
    Fg = out["forces"].cpu().numpy()
    del out
    m.close()
    dEi = Ea[cents] - e_ref
    dF = Fg[atoms] - F_ref
    frms = float(np.sqrt((F_ref ** 2).mean()))
    _report(f"subdomain_{'fp32' if prec == FP32 else 'bf16_mixed'}", mean_dEi=float(abs(dEi.mean())),
            max_dEi=float(np.abs(dEi).max()), max_dF=float(np.abs(dF).max()),
            rms_dF=float(np.sqrt((dF ** 2).mean())), Frms=frms, centres=int(len(cents)), atoms=int(len(atoms)))
    if prec == FP32:
        assert abs(dEi.mean()) <= 1e-6 and np.abs(dEi).max() <= 1e-5
        assert np.abs(dF).max() <= 1e-4
    else:
        assert abs(dEi.mean()) <= 1e-3
        assert np.sqrt((dF ** 2).mean()) <= 0.01 * frms
