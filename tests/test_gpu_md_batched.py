"""GPU tests of batched independent systems and of the FP64 velocity-Verlet
driver (eager and HIP-graph replay), through the C interface."""
import copy

import numpy as np
import pytest
import torch

import paper_2304_10061_amd as P
import workloads as W
from oracle import md as OMD
from oracle import model as OM
from oracle.neighbors import neighbor_list

from gpu_helpers import gpu_model, to_dev

pytestmark = pytest.mark.gpu

FP32, BF16 = P.PREC_FP32, P.PREC_BF16


def _cluster_batch():
    return W.clusters(10, 17, lo=20, hi=250)


@pytest.mark.parametrize("extras", [False, True], ids=["plain", "pair_cutoffs_zbl"])
def test_batched_neighbors_and_energies_equal_individual(extras):
    mc = W.model_config(5)
    if extras:   # the paper's ordered pair cutoffs and the ZBL term
        mc.pair_cutoffs = W.paper_pair_cutoffs(mc.n_species, mc.r_cut)
        mc.atomic_numbers = W.atomic_numbers(mc.n_species)
    w = W.make_weights(mc, np.random.default_rng(4))
    sc, sh = W.species_scale_shift(mc, np.random.default_rng(5))
    b = _cluster_batch()
    off = b.atom_offsets
    m = gpu_model(mc, w, FP32, sc, sh)
    pos, sp = to_dev(b)
    m.neighbors_batched(off, pos, sp)
    ci, nj, shf = m.copy_edges()
    ci, nj = ci.cpu().numpy(), nj.cpu().numpy()
    dev = pos.device
    n = b.n_total
    F = torch.empty((n, 3), dtype=torch.float64, device=dev)
    Ea = torch.empty(n, dtype=torch.float64, device=dev)
    Es = torch.empty(len(off) - 1, dtype=torch.float64, device=dev)
    m.energy_forces(pos, sp, F, atom_energy=Ea)
    m.system_energies(Ea, Es)
    torch.cuda.synchronize()
    F, Ea, Es = F.cpu().numpy(), Ea.cpu().numpy(), Es.cpu().numpy()
    edges = []
    for k in range(len(off) - 1):
        a, z = int(off[k]), int(off[k + 1])
        sub = W.System(pos=b.pos[a:z], species=b.species[a:z], cell=np.zeros(3), pbc=np.zeros(3, np.int32),
                       n_local=z - a)
        ri, rj, rs = neighbor_list(sub.pos, sub.cell, sub.pbc, mc.r_cut, species=sub.species,
                                   pair_cutoffs=mc.pair_cutoffs)
        edges.append((ri + a, rj + a))
        ref = OM.evaluate(mc, w, sub, sc, sh)
        assert abs(Es[k] - ref.energy) / (z - a) < 1e-6
        assert np.abs(F[a:z] - ref.forces).max() < 1e-4
        assert np.abs(Ea[a:z] - ref.atom_energy).max() < 1e-5
    assert np.array_equal(ci, np.concatenate([e[0] for e in edges]))
    assert np.array_equal(nj, np.concatenate([e[1] for e in edges]))
    assert np.all(shf.cpu().numpy() == 0)


def _md_setup(prec, skin=1.0, steps_model=1):
    mc, s, w = W.workload(1)
    m = P.Model(P.config_from(mc, precision=prec, neighbor_skin=skin), W.pack_weights(mc, w))
    v0 = W.maxwell_boltzmann(s.masses, 300.0, W.seeds(1)[4])
    return mc, s, w, m, v0


def _md_arrays(s, v0):
    dev = torch.device("cuda", 0)
    pos, sp = to_dev(s)
    vel = torch.as_tensor(v0, dtype=torch.float64, device=dev)
    masses = torch.as_tensor(s.masses, dtype=torch.float64, device=dev)
    F = torch.zeros((s.n_total, 3), dtype=torch.float64, device=dev)
    return pos, sp, vel, masses, F


def test_md_graph_replay_equals_eager():
    mc, s, w, m, v0 = _md_setup(FP32)
    runs = []
    for use_graph in (False, True):
        pos, sp, vel, masses, F = _md_arrays(s, v0)
        m.neighbors(pos, sp, s.cell, s.pbc)
        thermo = torch.zeros((10, 2), dtype=torch.float64, device=pos.device)
        m.md_run(5, 0.5, masses, pos, vel, F, sp, thermo=thermo, init_forces=True, use_graph=use_graph)
        # eager work between replays, then more replays of the same graph
        _ = (pos * 2.0).sum().item()
        m.md_run(5, 0.5, masses, pos, vel, F, sp, thermo=thermo[5:], use_graph=use_graph)
        torch.cuda.synchronize()
        runs.append((pos.cpu().numpy(), vel.cpu().numpy(), thermo.cpu().numpy()))
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)


def test_md_matches_oracle_short_run_and_conserves_energy():
    mc, s, w, m, v0 = _md_setup(FP32)
    pos, sp, vel, masses, F = _md_arrays(s, v0)
    m.neighbors(pos, sp, s.cell, s.pbc)
    n_steps, dt = 20, 0.25
    thermo = torch.zeros((n_steps, 2), dtype=torch.float64, device=pos.device)
    disp = m.md_run(n_steps, dt, masses, pos, vel, F, sp, thermo=thermo, init_forces=True)
    torch.cuda.synchronize()
    assert disp < 0.5
    p = OM.Params(mc, w)

    def ff(x):
        s2 = copy.copy(s)
        s2.pos = x
        r = OM.evaluate(mc, w, s2, params=p, need_atom_virial=False)
        return r.energy, r.forces

    xr, vr, et = OMD.velocity_verlet(ff, s.pos, v0, s.masses, dt, n_steps)
    # FP32 forces vs FP64 over 20 steps: trajectories still agree closely
    assert np.abs(pos.cpu().numpy() - xr).max() < 1e-6
    th = thermo.cpu().numpy()
    etot = th[:, 0] + th[:, 1]
    assert np.abs(etot - et[1:]).max() < 1e-4
    assert np.abs(etot - etot[0]).max() < 1e-3


def test_md_ghost_shell_equals_periodic():
    mc = W.model_config(4)
    w = W.make_weights(mc, np.random.default_rng(3))
    base = W.jittered_lattice_box(1000, (1000 / 0.1) ** (1 / 3), 0.5, W.PROTEIN_MIX, 31)
    g = W.ghost_shell(base, 6.0)
    v0 = W.maxwell_boltzmann(base.masses, 300.0, W.seeds(4)[4])
    out = []
    for sysm in (base, g):
        m = P.Model(P.config_from(mc, precision=FP32, neighbor_skin=1.0), W.pack_weights(mc, w))
        pos, sp = to_dev(sysm)
        dev = pos.device
        vel = torch.as_tensor(v0, dtype=torch.float64, device=dev)
        masses = torch.as_tensor(base.masses, dtype=torch.float64, device=dev)
        F = torch.zeros((sysm.n_total, 3), dtype=torch.float64, device=dev)
        if sysm is g:
            own = g.ghost_owner
            m.set_ghosts(base.n_local, own, g.pos[base.n_local:] - base.pos[own])
        m.neighbors(pos, sp, sysm.cell, sysm.pbc, sysm.n_local)
        thermo = torch.zeros((10, 2), dtype=torch.float64, device=dev)
        m.md_run(10, 0.5, masses, pos, vel, F, sp, thermo=thermo, init_forces=True)
        torch.cuda.synchronize()
        out.append((pos[:base.n_local].cpu().numpy(), thermo.cpu().numpy()))
    # same dynamics; only FP32 summation order differs (ghost images vs shifts)
    assert np.abs(out[0][0] - out[1][0]).max() < 1e-6
    assert np.abs(out[0][1] - out[1][1]).max() < 1e-4
