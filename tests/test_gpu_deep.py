"""Deeper tensor tracks on the HIP path against the FP64 oracle: three and four
layers (unnatural-parity irreps in the middle layers, triple-product
couplings, per-irrep mixing) and l_max = 3 (l = 3 harmonics, wider coupling
tables).  Tolerances as in the other parity tests:
  FP32         |E - E_ref| / N <= 1e-6 eV/atom, max |F - F_ref| <= 1e-4 eV/A
  BF16-mixed   |E - E_ref| / N <= 1e-3 eV/atom, RMS(F - F_ref) <= 1% of RMS(F_ref)
The 3,000-atom water box with the three-layer l_max 3 model is checked on
sampled centres (their atom energies) and sampled atoms (their forces), each
computed by the oracle from the centres' own edges.
"""
import copy

import numpy as np
import pytest

import paper_2304_10061_amd as P
import workloads as W
from oracle import model as OM
from oracle.neighbors import neighbor_list

from gpu_helpers import gpu_eval, gpu_model
from gpu_helpers import sampled_reference as _sampled_reference
from test_gpu_parity import _check_bf16, _check_fp32, _report

pytestmark = pytest.mark.gpu

FP32, BF16M = P.PREC_FP32, P.PREC_BF16_MIXED

DEEP = [
    ("l2_three_layers", dict(l_max=2, n_layers=3, n_tensor=32)),
    ("l3_three_layers", dict(l_max=3, n_layers=3, n_tensor=32)),
    ("l3_two_layers_n64", dict(l_max=3, n_layers=2, n_tensor=64)),
    ("l3_one_layer", dict(l_max=3, n_layers=1, n_tensor=32)),
    ("l1_four_layers", dict(l_max=1, n_layers=4, n_tensor=32)),
    ("l2_four_layers_n64", dict(l_max=2, n_layers=4, n_tensor=64)),
    ("l3_three_layers_no_mix", dict(l_max=3, n_layers=3, n_tensor=32, channel_mix=False)),
    # the largest pattern (both parities in and out, 1191 non-zeros) with 64 channels
    ("l3_four_layers_n64", dict(l_max=3, n_layers=4, n_tensor=64)),
]


def _small(kw):
    return W.ModelConfig(n_species=2, r_cut=4.0, twobody_dims=(64, 64), latent_dims=(64, 64), **kw)


@pytest.mark.parametrize("case", DEEP, ids=lambda c: c[0])
@pytest.mark.parametrize("prec", [FP32, BF16M], ids=["fp32", "bf16_mixed"])
def test_deep_small_models(case, prec):
    name, kw = case
    mc = _small(kw)
    w = W.make_weights(mc, np.random.default_rng(31))
    s = W.system(1)
    sc, sh = W.species_scale_shift(mc, np.random.default_rng(32))
    ref = OM.evaluate(mc, w, s, sc, sh)
    print("case", name, "prec", prec, flush=True)
    got = gpu_eval(gpu_model(mc, w, prec, sc, sh), s)
    if prec == FP32:
        _check_fp32(f"{name}_fp32", got, ref, s.n_local)
        assert np.abs(got["atom_energy"] - ref.atom_energy).max() < 1e-5
    else:
        _check_bf16(f"{name}_bf16_mixed", got, ref, s.n_local)


def test_deep_with_pair_cutoffs_and_zbl():
    mc = _small(dict(l_max=3, n_layers=3, n_tensor=32))
    mc.pair_cutoffs = W.paper_pair_cutoffs(2, mc.r_cut)
    mc.atomic_numbers = W.atomic_numbers(2)
    w = W.make_weights(mc, np.random.default_rng(33))
    s = W.system(1)
    ref = OM.evaluate(mc, w, s)
    got = gpu_eval(gpu_model(mc, w, FP32), s)
    _check_fp32("l3_three_layers_pairs_zbl_fp32", got, ref, s.n_local)


def test_deep_chunked_equals_whole():
    """Chunks start at arbitrary edge offsets, so every kernel must round an
    edge's arithmetic the same wherever the edge sits in a tile."""
    mc = _small(dict(l_max=3, n_layers=3, n_tensor=32))
    w = W.make_weights(mc, np.random.default_rng(34))
    s = W.system(1)
    a = gpu_eval(gpu_model(mc, w, FP32), s)
    b = gpu_eval(gpu_model(mc, w, FP32, edge_chunk=300), s)
    _report("deep_chunked", max_dF=float(np.abs(a["forces"] - b["forces"]).max()),
            n_diff=int((a["forces"] != b["forces"]).sum()))
    assert np.array_equal(a["forces"], b["forces"])
    assert np.array_equal(a["atom_energy"], b["atom_energy"])


def test_deep_mirror_image():
    """Mirror-imaged positions give the same energies and mirrored forces on
    the GPU too (a wrongly assigned parity would leave a pseudoscalar)."""
    mc = _small(dict(l_max=3, n_layers=3, n_tensor=32))
    w = W.make_weights(mc, np.random.default_rng(35))
    s = W.clusters(3, 9, ratio=W.WATER_MIX)
    s2 = copy.copy(s)
    s2.pos = s.pos * np.array([-1.0, 1.0, 1.0])
    a = gpu_eval(gpu_model(mc, w, FP32), s)
    b = gpu_eval(gpu_model(mc, w, FP32), s2)
    _report("mirror", dE=float(abs(a["energy"][0] - b["energy"][0])),
            max_dF=float(np.abs(b["forces"] - a["forces"] * np.array([-1.0, 1.0, 1.0])).max()))
    assert abs(float(a["energy"][0] - b["energy"][0])) <= 1e-6 * s.n_local
    assert np.abs(b["forces"] - a["forces"] * np.array([-1.0, 1.0, 1.0])).max() <= 1e-4


@pytest.fixture(scope="module")
def deep_box():
    mc, s, w = W.deep_workload()
    nbr = neighbor_list(s.pos, s.cell, s.pbc, mc.r_cut, method="kdtree")
    return mc, s, w, nbr


@pytest.mark.parametrize("prec", [FP32, BF16M], ids=["fp32", "bf16_mixed"])
def test_deep_water_box_sampled(deep_box, prec):
    mc, s, w, nbr = deep_box
    got = gpu_eval(gpu_model(mc, w, prec), s, want_atom_virial=False)
    cents, e_ref, atoms, F_ref = _sampled_reference(mc, s, w, nbr, np.random.default_rng(7))
    dEi = got["atom_energy"][cents] - e_ref
    dF = got["forces"][atoms] - F_ref
    frms = float(np.sqrt((F_ref ** 2).mean()))
    _report(f"deep_box_{'fp32' if prec == FP32 else 'bf16_mixed'}", mean_dEi=float(abs(dEi.mean())),
            max_dEi=float(np.abs(dEi).max()), max_dF=float(np.abs(dF).max()), Frms=frms)
    if prec == FP32:
        assert abs(dEi.mean()) <= 1e-6 and np.abs(dEi).max() <= 1e-5
        assert np.abs(dF).max() <= 1e-4
    else:
        assert abs(dEi.mean()) <= 1e-3
        assert np.sqrt((dF ** 2).mean()) <= 0.01 * frms
    assert np.abs(got["forces"].sum(0)).max() < 1e-6 * s.n_local


def test_deep_md_graph_replay_and_oracle_trajectory():
    """FP64 velocity Verlet with a deep model: hipGraph replays equal eager
    steps bit for bit, and a short trajectory follows the oracle's."""
    import torch
    from oracle import md as OMD
    from test_gpu_md_batched import _md_arrays
    mc = _small(dict(l_max=3, n_layers=3, n_tensor=32))
    w = W.make_weights(mc, np.random.default_rng(36))
    s = W.system(1)
    m = P.Model(P.config_from(mc, precision=FP32, neighbor_skin=1.0), W.pack_weights(mc, w))
    v0 = W.maxwell_boltzmann(s.masses, 300.0, np.random.default_rng(37))
    n_steps, dt = 10, 0.25
    runs = []
    for use_graph in (False, True):
        pos, sp, vel, masses, F = _md_arrays(s, v0)
        m.neighbors(pos, sp, s.cell, s.pbc)
        thermo = torch.zeros((n_steps, 2), dtype=torch.float64, device=pos.device)
        m.md_run(n_steps, dt, masses, pos, vel, F, sp, thermo=thermo, init_forces=True, use_graph=use_graph)
        torch.cuda.synchronize()
        runs.append((pos.cpu().numpy(), vel.cpu().numpy(), thermo.cpu().numpy()))
    for a, b in zip(runs[0], runs[1]):
        assert np.array_equal(a, b)
    p = OM.Params(mc, w)

    def ff(x):
        s2 = copy.copy(s)
        s2.pos = x
        r = OM.evaluate(mc, w, s2, params=p, need_atom_virial=False)
        return r.energy, r.forces

    xr, vr, et = OMD.velocity_verlet(ff, s.pos, v0, s.masses, dt, n_steps)
    _report("deep_md", max_dx=float(np.abs(runs[0][0] - xr).max()))
    assert np.abs(runs[0][0] - xr).max() < 1e-6
    etot = runs[0][2][:, 0] + runs[0][2][:, 1]
    assert np.abs(etot - et[1:]).max() < 1e-4


@pytest.mark.parametrize("prec", [FP32, BF16M], ids=["fp32", "bf16_mixed"])
def test_deep_empty_isolated_and_dimer(prec):
    """Degenerate inputs with a deep model: no atoms, isolated atoms (energy =
    species shift, zero force), and a single pair (every edge in one centre
    segment, the tile mostly padding) against the oracle."""
    mc = _small(dict(l_max=3, n_layers=3, n_tensor=32))
    w = W.make_weights(mc, np.random.default_rng(38))
    sc, sh = W.species_scale_shift(mc, np.random.default_rng(39))
    m = gpu_model(mc, w, prec, sc, sh)
    s0 = W.System(pos=np.zeros((0, 3)), species=np.zeros(0, np.int32), cell=np.zeros(3),
                  pbc=np.zeros(3, np.int32), n_local=0)
    assert gpu_eval(m, s0)["energy"][0] == 0.0
    iso = W.System(pos=np.array([[0.0, 0.0, 0.0], [10.0, 0.0, 0.0]]), species=np.array([0, 1], np.int32),
                   cell=np.zeros(3), pbc=np.zeros(3, np.int32), n_local=2)
    got = gpu_eval(m, iso)
    assert np.all(got["forces"] == 0.0)
    assert np.allclose(got["atom_energy"], sh[[0, 1]])
    dimer = W.System(pos=np.array([[0.0, 0.0, 0.0], [1.3, 0.4, -0.2]]), species=np.array([1, 0], np.int32),
                     cell=np.zeros(3), pbc=np.zeros(3, np.int32), n_local=2)
    ref = OM.evaluate(mc, w, dimer, sc, sh)
    got = gpu_eval(m, dimer)
    if prec == FP32:
        _check_fp32("deep_dimer_fp32", got, ref, 2)
    else:
        _check_bf16("deep_dimer_bf16_mixed", got, ref, 2)
