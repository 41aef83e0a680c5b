"""The ZBL repulsive pair term (section "Training details") on the HIP path
against the FP64 oracle: FP32 and BF16-mixed energies, forces and virial on the
water box (H = 1, O = 8), combined with the paper's ordered pair cutoffs, and
a close dimer whose energy is the pair term alone (silent network).
"""
import copy

import numpy as np
import pytest

import paper_2304_10061_amd as P
import workloads as W
from oracle import model as OM

from gpu_helpers import gpu_eval, gpu_model
from test_gpu_parity import _check_bf16, _check_fp32, _report

pytestmark = pytest.mark.gpu


def with_zbl(mc, pairs=False):
    m = copy.copy(mc)
    m.atomic_numbers = W.atomic_numbers(mc.n_species)
    if pairs:
        m.pair_cutoffs = W.paper_pair_cutoffs(mc.n_species, mc.r_cut)
    return m


@pytest.fixture(scope="module", params=[False, True], ids=["single_cutoff", "pair_cutoffs"])
def water_zbl(request):
    mc, s, w = W.workload(2)
    mc = with_zbl(mc, request.param)
    sc, sh = W.species_scale_shift(mc, np.random.default_rng(21))
    ref = OM.evaluate(mc, w, s, sc, sh)
    return request.param, mc, s, w, sc, sh, ref


def test_zbl_fp32_water_box(water_zbl):
    pairs, mc, s, w, sc, sh, ref = water_zbl
    got = gpu_eval(gpu_model(mc, w, P.PREC_FP32, sc, sh), s)
    _check_fp32(f"cfg2_zbl{'_pairs' if pairs else ''}_fp32", got, ref, s.n_local)
    assert np.abs(got["atom_energy"] - ref.atom_energy).max() < 1e-5


def test_zbl_bf16_mixed_water_box(water_zbl):
    pairs, mc, s, w, sc, sh, ref = water_zbl
    got = gpu_eval(gpu_model(mc, w, P.PREC_BF16_MIXED, sc, sh), s)
    _check_bf16(f"cfg2_zbl{'_pairs' if pairs else ''}_bf16_mixed", got, ref, s.n_local)


def test_zbl_close_dimer_silent_network():
    mc = with_zbl(W.model_config(2))
    w = {k: np.zeros_like(v) for k, v in W.make_weights(mc, np.random.default_rng(3)).items()}
    for d in (0.55, 1.1, 2.2):
        pos = np.array([[5.0, 5.0, 5.0], [5.0 + d, 5.0, 5.0]])
        s = W.System(pos=pos, species=np.array([1, 0], np.int32), cell=np.zeros(3), pbc=np.zeros(3, np.int32),
                     n_local=2)
        ref = OM.evaluate(mc, w, s)
        got = gpu_eval(gpu_model(mc, w, P.PREC_FP32), s)
        e, f = float(got["energy"][0]), got["forces"]
        _report("zbl_dimer", d=d, energy=e, ref=ref.energy, force=float(f[1, 0]), ref_force=float(ref.forces[1, 0]))
        assert abs(e - ref.energy) <= 2e-6 * max(1.0, abs(ref.energy))
        assert np.abs(f - ref.forces).max() <= 2e-6 * max(1.0, float(np.abs(ref.forces).max()))


def test_md_with_pair_cutoffs_and_zbl_matches_oracle():
    """Short NVE run of the 64-atom box with the paper's pair cutoffs and the
    ZBL term, hipGraph-replayed on the GPU, against the oracle's FP64
    velocity Verlet: positions and total energy track, and energy is kept."""
    import torch
    from oracle import md as OMD
    from gpu_helpers import to_dev
    mc, s, w = W.workload(1)
    mc = with_zbl(mc, pairs=True)
    m = P.Model(P.config_from(mc, precision=P.PREC_FP32, neighbor_skin=1.0), W.pack_weights(mc, w))
    v0 = W.maxwell_boltzmann(s.masses, 300.0, W.seeds(1)[4])
    pos, sp = to_dev(s)
    dev = pos.device
    vel = torch.as_tensor(v0, dtype=torch.float64, device=dev)
    masses = torch.as_tensor(s.masses, dtype=torch.float64, device=dev)
    F = torch.zeros((s.n_total, 3), dtype=torch.float64, device=dev)
    m.neighbors(pos, sp, s.cell, s.pbc)
    n_steps, dt = 20, 0.25
    thermo = torch.zeros((n_steps, 2), dtype=torch.float64, device=dev)
    disp = m.md_run(n_steps, dt, masses, pos, vel, F, sp, thermo=thermo, init_forces=True, use_graph=True)
    torch.cuda.synchronize()
    assert disp < 0.5
    p = OM.Params(mc, w)

    def ff(x):
        s2 = copy.copy(s)
        s2.pos = x
        r = OM.evaluate(mc, w, s2, params=p, need_atom_virial=False)
        return r.energy, r.forces

    xr, vr, et = OMD.velocity_verlet(ff, s.pos, v0, s.masses, dt, n_steps)
    th = thermo.cpu().numpy()
    etot = th[:, 0] + th[:, 1]
    _report("md_pairs_zbl", max_dx=float(np.abs(pos.cpu().numpy() - xr).max()),
            max_dE=float(np.abs(etot - et[1:]).max()), drift=float(np.abs(etot - etot[0]).max()))
    assert np.abs(pos.cpu().numpy() - xr).max() < 1e-6
    assert np.abs(etot - et[1:]).max() < 1e-4
    # energy is kept as well as the FP64 integrator keeps it at this time step
    assert np.abs(etot - etot[0]).max() < np.abs(et - et[0]).max() + 1e-4
