"""GPU tests of the neighbour-list rebuild inside allegro_md_run: rebuilds on
the device within a fixed edge capacity (eager and HIP-graph replay give the
same bits), agreement with the FP64 oracle's velocity Verlet, which rebuilds
its neighbour list at every step, and the capacity overflow path
(ALLEGRO_E_CAPACITY, regrowth, resumption on the same trajectory)."""
import copy

import numpy as np
import pytest
import torch

import paper_2304_10061_amd as P
import workloads as W
from oracle import md as OMD
from oracle import model as OM

from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu

FP32, MIXED = P.PREC_FP32, P.PREC_BF16_MIXED
CAPACITY = -3


def _model(mc, w, prec, skin, hint=0, edge_chunk=0):
    cfg = P.config_from(mc, precision=prec, neighbor_skin=skin, edge_capacity_hint=hint, edge_chunk=edge_chunk)
    return P.Model(cfg, W.pack_weights(mc, w))


def _state(s, v0, F0=None):
    dev = torch.device("cuda", 0)
    pos, sp = to_dev(s)
    vel = torch.as_tensor(v0, dtype=torch.float64, device=dev)
    masses = torch.as_tensor(s.masses, dtype=torch.float64, device=dev)
    F = torch.zeros((s.n_total, 3), dtype=torch.float64, device=dev) if F0 is None else F0.clone()
    return pos, sp, vel, masses, F


def _host(*ts):
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ts]


@pytest.mark.parametrize("prec", [FP32, MIXED], ids=["fp32", "bf16_mixed"])
def test_graph_steps_with_device_rebuilds_equal_eager_steps(prec):
    """40 steps of the 3,000-atom water box with a 0.1 A skin: the list is
    rebuilt on the device many times; one captured step replayed 40 times
    (over two calls, one capture) gives the bits of 40 eager steps."""
    mc, s, w = W.workload(2)
    v0 = W.maxwell_boltzmann(s.masses, 300.0, W.seeds(2)[4])
    runs, stats = [], []
    for use_graph in (False, True):
        # the jittered box relaxes and gains edges: capacity for twice the start
        m = _model(mc, w, prec, skin=0.1, hint=160000)
        pos, sp, vel, masses, F = _state(s, v0)
        m.neighbors(pos, sp, s.cell, s.pbc)
        thermo = torch.zeros((20, 2), dtype=torch.float64, device=pos.device)
        m.md_run(20, 0.5, masses, pos, vel, F, sp, thermo=thermo, init_forces=True, use_graph=use_graph)
        nb1 = m.md_stats()[3]
        th1 = thermo.clone()
        _ = (pos * 2.0).sum().item()   # eager work between the calls
        m.md_run(20, 0.5, masses, pos, vel, F, sp, thermo=thermo, use_graph=use_graph)
        caps, cap, dev, nb2 = m.md_stats()
        runs.append(_host(pos, vel, F, th1, thermo))
        stats.append((caps, dev, nb1, nb2))
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)
    (caps_e, dev_e, nb1_e, nb2_e), (caps_g, dev_g, nb1_g, nb2_g) = stats
    assert dev_e == 1 and dev_g == 1
    assert caps_e == 0 and caps_g == 1            # 40 replays of one capture
    assert (nb1_e, nb2_e) == (nb1_g, nb2_g)
    assert nb1_e >= 3 and nb2_e >= 3              # the device did rebuild


def test_device_rebuilds_follow_oracle_trajectory():
    """FP32 steps with a 0.05 A skin (rebuilt on the device every few steps)
    against the FP64 oracle, whose neighbour list is rebuilt every step."""
    mc, s, w = W.workload(1)
    v0 = W.maxwell_boltzmann(s.masses, 300.0, W.seeds(1)[4])
    m = _model(mc, w, FP32, skin=0.05, hint=8000)
    pos, sp, vel, masses, F = _state(s, v0)
    m.neighbors(pos, sp, s.cell, s.pbc)
    n_steps, dt = 24, 0.25
    thermo = torch.zeros((n_steps, 2), dtype=torch.float64, device=pos.device)
    m.md_run(n_steps, dt, masses, pos, vel, F, sp, thermo=thermo, init_forces=True, use_graph=True)
    caps, cap, dev, nb = m.md_stats()
    assert dev == 1 and nb >= 2
    p = OM.Params(mc, w)

    def ff(x):
        s2 = copy.copy(s)
        s2.pos = x
        r = OM.evaluate(mc, w, s2, params=p, need_atom_virial=False)
        return r.energy, r.forces

    xr, vr, et = OMD.velocity_verlet(ff, s.pos, v0, s.masses, dt, n_steps)
    x, th = _host(pos, thermo)
    assert np.abs(x - xr).max() < 1e-6
    assert np.abs(th[:, 0] + th[:, 1] - et[1:]).max() < 1e-4


def test_host_rebuilds_of_chunked_lists_match_device_rebuilds():
    """A list split over several evaluation chunks is rebuilt by the host
    between eager steps; per-edge and per-centre results do not depend on the
    chunking, so the trajectory is the device-rebuild one."""
    mc, s, w = W.workload(2)
    v0 = W.maxwell_boltzmann(s.masses, 300.0, W.seeds(2)[4])
    out = []
    for chunk in (0, 30000):
        m = _model(mc, w, FP32, skin=0.1, hint=160000, edge_chunk=chunk)
        pos, sp, vel, masses, F = _state(s, v0)
        m.neighbors(pos, sp, s.cell, s.pbc)
        m.md_run(16, 0.5, masses, pos, vel, F, sp, init_forces=True, use_graph=True)
        out.append((_host(pos, vel, F), m.md_stats()))
    (a, st_dev), (b, st_host) = out
    assert st_dev[2] == 1 and st_host[2] == 0
    assert st_host[0] == 0                        # no graph for host rebuilds
    assert st_dev[3] == st_host[3] and st_dev[3] >= 2
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-9 * max(1.0, np.abs(x).max())


def test_batched_clusters_graph_rebuilds_equal_eager():
    """Uneven non-periodic clusters in one batched list (each system binned
    in its own slot of the cell grid), rebuilt on the device inside the step:
    graph replays give the eager steps' bits, and the rebuilt lists keep
    every system's pairs to itself."""
    mc = W.model_config(5)
    w = W.make_weights(mc, np.random.default_rng(4))
    b = W.clusters(12, 21, lo=20, hi=300)
    v0 = W.maxwell_boltzmann(b.masses, 300.0, np.random.default_rng(22))
    out, stats = [], []
    for use_graph in (False, True):
        m = _model(mc, w, MIXED, skin=0.1, hint=4 * 30 * b.n_local)
        pos, sp, vel, masses, F = _state(b, v0)
        m.neighbors_batched(b.atom_offsets, pos, sp)
        thermo = torch.zeros((24, 2), dtype=torch.float64, device=pos.device)
        m.md_run(24, 0.5, masses, pos, vel, F, sp, thermo=thermo, init_forces=True, use_graph=use_graph)
        stats.append(m.md_stats())
        ci, nj, _ = m.copy_edges()
        ci, nj = _host(ci, nj)
        sysid = np.searchsorted(b.atom_offsets, np.arange(b.n_local), side="right") - 1
        assert np.array_equal(sysid[ci], sysid[nj])
        out.append(_host(pos, vel, F, thermo))
    for a_, b_ in zip(out[0], out[1]):
        assert np.array_equal(a_, b_)
    assert stats[0][2] == 1 and stats[0][3] >= 2 and stats[0][3] == stats[1][3]
    assert stats[1][0] == 1


def test_ghost_shell_with_device_rebuilds_matches_periodic_box():
    """One GPU's share with its ghost shell (non-periodic, ghosts following
    their owners) against the periodic box, with a 0.1 A skin so that the
    device rebuilds the lists during the run: the same trajectory up to FP32
    summation order."""
    mc = W.model_config(4)
    w = W.make_weights(mc, np.random.default_rng(3))
    base = W.jittered_lattice_box(1000, (1000 / 0.1) ** (1 / 3), 0.5, W.PROTEIN_MIX, 31)
    g = W.ghost_shell(base, 6.0)
    v0 = W.maxwell_boltzmann(base.masses, 300.0, W.seeds(4)[4])
    res = []
    for sysm in (base, g):
        m = _model(mc, w, FP32, skin=0.1, hint=60 * sysm.n_total)
        pos, sp = to_dev(sysm)
        dev = pos.device
        vel = torch.as_tensor(v0, dtype=torch.float64, device=dev)
        masses = torch.as_tensor(base.masses, dtype=torch.float64, device=dev)
        F = torch.zeros((sysm.n_total, 3), dtype=torch.float64, device=dev)
        if sysm is g:
            own = g.ghost_owner
            m.set_ghosts(base.n_local, own, g.pos[base.n_local:] - base.pos[own])
        m.neighbors(pos, sp, sysm.cell, sysm.pbc, sysm.n_local)
        thermo = torch.zeros((20, 2), dtype=torch.float64, device=dev)
        m.md_run(20, 0.5, masses, pos, vel, F, sp, thermo=thermo, init_forces=True, use_graph=True)
        assert m.md_stats()[2] == 1 and m.md_stats()[3] >= 2
        res.append((_host(pos)[0][:base.n_local], _host(thermo)[0]))
    assert np.abs(res[0][0] - res[1][0]).max() < 1e-6
    assert np.abs(res[0][1] - res[1][1]).max() < 1e-4


def test_per_step_virial_rows():
    """The per-step virial of allegro_md_run: graph replays give the eager
    rows bit for bit, and the last row is the virial allegro_energy_forces
    reports at the final positions (the last half kick moves no atom)."""
    mc, s, w = W.workload(2)
    v0 = W.maxwell_boltzmann(s.masses, 300.0, W.seeds(2)[4])
    rows = []
    for use_graph in (False, True):
        m = _model(mc, w, FP32, skin=0.1, hint=160000)
        pos, sp, vel, masses, F = _state(s, v0)
        m.neighbors(pos, sp, s.cell, s.pbc)
        vir = torch.full((12, 9), float("nan"), dtype=torch.float64, device=pos.device)
        m.md_run(12, 0.5, masses, pos, vel, F, sp, virial=vir, init_forces=True, use_graph=use_graph)
        rows.append(_host(vir)[0])
        assert m.md_stats()[3] >= 1
        F2 = torch.empty_like(F)
        v_now = torch.empty(9, dtype=torch.float64, device=pos.device)
        m.energy_forces(pos, sp, F2, virial=v_now)
        last, ef = _host(vir[-1], v_now)
        assert np.allclose(last, ef, rtol=1e-12, atol=1e-12)
    assert np.all(np.isfinite(rows[0]))
    assert np.array_equal(rows[0], rows[1])
    # an invariant model's virial is symmetric (FP32 sums)
    W3 = rows[0].reshape(-1, 3, 3)
    assert np.abs(W3 - W3.transpose(0, 2, 1)).max() <= 1e-5 * np.abs(W3).max()


@pytest.mark.parametrize("prec", [FP32, MIXED], ids=["fp32", "bf16_mixed"])
def test_capacity_overflow_regrows_and_resumes_on_the_same_trajectory(prec):
    """The list is first built on the unjittered lattice (about 23 neighbours
    per atom within 4.1 A) and the run starts from the jittered box (about
    26): with the capacity of the lattice list (hint 1) the first device
    rebuild overflows.  allegro_md_run discards the step, regrows, and the resumed
    run matches a run with ample capacity bit for bit."""
    mc, s, w = W.workload(2)
    lat = W.jittered_lattice_box(s.n_local, float(s.cell[0]), 0.0, W.WATER_MIX, 2, sites_per_side=15)
    v0 = W.maxwell_boltzmann(s.masses, 300.0, W.seeds(2)[4])
    n_steps, dt, skin = 30, 0.5, 0.1
    # forces at the start, from a list built at the start
    m0 = _model(mc, w, prec, skin=skin)
    pos0, sp = to_dev(s)
    F0 = m0.evaluate(pos0, sp, s.cell, s.pbc)["forces"].clone()
    lat_pos = torch.as_tensor(lat.pos, dtype=torch.float64, device=pos0.device)

    ref = _model(mc, w, prec, skin=skin, hint=200000)
    pos, sp, vel, masses, F = _state(s, v0, F0)
    ref.neighbors(lat_pos, sp, s.cell, s.pbc)
    e_lat = ref.num_edges()
    thermo_r = torch.zeros((n_steps, 2), dtype=torch.float64, device=pos.device)
    ref.md_run(n_steps, dt, masses, pos, vel, F, sp, thermo=thermo_r, use_graph=True)
    want = _host(pos, vel, F, thermo_r)
    assert ref.md_stats()[1] == 200000 and ref.md_stats()[3] >= 3

    tiny = _model(mc, w, prec, skin=skin, hint=1)
    pos, sp, vel, masses, F = _state(s, v0, F0)
    tiny.neighbors(lat_pos, sp, s.cell, s.pbc)
    assert tiny.md_stats()[1] == e_lat            # the capacity is the lattice list
    thermo = torch.zeros((n_steps, 2), dtype=torch.float64, device=pos.device)
    done, overflows, caps = 0, [], []
    for _ in range(10):
        try:
            tiny.md_run(n_steps - done, dt, masses, pos, vel, F, sp, thermo=thermo[done:], use_graph=True)
            break
        except P.AllegroError as e:
            assert e.status == CAPACITY
            overflows.append(e.steps_done)
            caps.append(tiny.md_stats()[1])
            done += e.steps_done
    else:
        pytest.fail("the run kept overflowing")
    assert overflows and overflows[0] == 0        # the first rebuild is at the first step
    assert caps[0] > e_lat and caps == sorted(caps)
    got = _host(pos, vel, F, thermo)
    for a, b in zip(want, got):
        assert np.array_equal(a, b)
