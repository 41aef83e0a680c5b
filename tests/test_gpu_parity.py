"""Parity of the HIP path (through the C interface) with the FP64 oracle.

Tolerances (FP64 oracle as reference):
  neighbour lists     bit-exact (i, j, shift) arrays
  FP32 path           |E - E_ref| / N <= 1e-6 eV/atom, max |F - F_ref| <= 1e-4 eV/A
  BF16-mixed path     |E - E_ref| / N <= 1e-3 eV/atom, RMS(F - F_ref) <= 1% of RMS(F_ref)
Inputs are the seeded synthetic workloads; the oracle never sees GPU output.
"""
import copy
import math

import numpy as np
import pytest
import torch

import paper_2304_10061_amd as P
import workloads as W
from oracle import model as OM
from oracle.neighbors import neighbor_list

from gpu_helpers import gpu_edges, gpu_eval, gpu_model, to_dev

pytestmark = pytest.mark.gpu

FP32, BF16, BF16S, BF16M = P.PREC_FP32, P.PREC_BF16, P.PREC_BF16_SINGLE, P.PREC_BF16_MIXED


def _report(tag, **kw):
    print(tag, " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in kw.items()), flush=True)


def _check_fp32(tag, got, ref, n):
    dE = abs(float(got["energy"][0]) - ref.energy) / n
    dF = float(np.abs(got["forces"] - ref.forces).max())
    dEi = float(np.abs(got["atom_energy"] - ref.atom_energy).max())
    dW = float(np.abs(got["virial"].reshape(3, 3) - ref.virial).max())
    _report(tag, dE_per_atom=dE, max_dF=dF, max_dEi=dEi, max_dW=dW, Frms=float(np.sqrt((ref.forces ** 2).mean())))
    assert dE <= 1e-6
    assert dF <= 1e-4
    assert dW <= 1e-4 * max(1.0, float(np.abs(ref.virial).max()))


def _check_bf16(tag, got, ref, n):
    dE = abs(float(got["energy"][0]) - ref.energy) / n
    rel = float(np.sqrt(((got["forces"] - ref.forces) ** 2).mean()) / np.sqrt((ref.forces ** 2).mean()))
    _report(tag, dE_per_atom=dE, force_rel_rms=rel)
    assert dE <= 1e-3
    assert rel <= 0.01


# ----------------------------------------------------------------------------- neighbours

def _nbr_cases():
    mc1, s1 = W.model_config(1), W.system(1)
    cases = [("cfg1", s1, 4.0), ("cfg2", W.system(2), 4.0)]
    g = W.ghost_shell(s1, 6.0)
    cases.append(("cfg1_ghosts", g, 4.0))
    un = copy.copy(s1)
    pos = s1.pos.copy()
    pos[::3] += np.array([8.6, -17.2, 25.8])        # unwrapped images of the same atoms
    un.pos = pos
    cases.append(("unwrapped", un, 4.0))
    tiny = W.System(pos=np.array([[0.5, 1.0, 2.0], [2.9, 0.1, 0.4], [1.5, 1.5, 1.5]]),
                    species=np.array([0, 1, 0], dtype=np.int32), cell=np.array([3.0, 3.0, 3.0]),
                    pbc=np.ones(3, np.int32), n_local=3)
    cases.append(("box_smaller_than_cutoff", tiny, 4.5))
    tie = W.System(pos=np.array([[1.0, 1.0, 1.0], [5.0, 1.0, 1.0], [1.0, 4.5, 1.0], [17.25, 1.0, 1.0]]),
                   species=np.zeros(4, np.int32), cell=np.array([20.0, 20.0, 20.0]),
                   pbc=np.ones(3, np.int32), n_local=4)
    cases.append(("exact_ties", tie, 4.0))
    mixed = copy.copy(W.system(2))
    mixed.pbc = np.array([1, 1, 0], np.int32)
    cases.append(("mixed_pbc", mixed, 4.0))
    cl = W.clusters(6, 11)
    cases.append(("clusters", cl, 4.0))
    ghosts_only_local = copy.copy(g)
    ghosts_only_local.n_local = 10
    cases.append(("few_centres", ghosts_only_local, 4.0))
    return cases


@pytest.mark.parametrize("case", _nbr_cases(), ids=lambda c: c[0])
def test_neighbors_bit_exact(case):
    name, s, rc = case
    mc = W.ModelConfig(n_species=4, r_cut=rc, l_max=1, n_layers=1, n_tensor=8,
                       twobody_dims=(32, 32), latent_dims=(32, 32))
    w = W.make_weights(mc, np.random.default_rng(0))
    m = gpu_model(mc, w, FP32)
    i, j, sh = gpu_edges(m, s)
    ri, rj, rs = neighbor_list(s.pos, s.cell, s.pbc, rc, n_local=s.n_local)
    _report(name, edges=len(ri))
    assert np.array_equal(i, ri) and np.array_equal(j, rj) and np.array_equal(sh, rs)


def test_neighbors_bit_exact_protein_box():
    mc = W.model_config(3)
    s = W.system(3)
    m = gpu_model(mc, W.make_weights(mc, np.random.default_rng(0)), BF16)
    i, j, sh = gpu_edges(m, s)
    ri, rj, rs = neighbor_list(s.pos, s.cell, s.pbc, mc.r_cut, method="kdtree")
    _report("cfg3", edges=len(ri), per_atom=len(ri) / s.n_local)
    assert np.array_equal(i, ri) and np.array_equal(j, rj) and np.array_equal(sh, rs)


# ----------------------------------------------------------------------------- energies/forces

@pytest.fixture(scope="module")
def cfg2():
    mc, s, w = W.workload(2)
    sc, sh = W.species_scale_shift(mc, np.random.default_rng(21))
    ref = OM.evaluate(mc, w, s, sc, sh)
    return mc, s, w, sc, sh, ref


def test_fp32_water_box(cfg2):
    mc, s, w, sc, sh, ref = cfg2
    m = gpu_model(mc, w, FP32, sc, sh)
    got = gpu_eval(m, s)
    _check_fp32("cfg2_fp32", got, ref, s.n_local)
    assert np.allclose(got["atom_virial"].reshape(-1, 3, 3).sum(0), got["virial"].reshape(3, 3), atol=1e-8)
    assert np.abs(got["atom_energy"] - ref.atom_energy).max() < 1e-5


@pytest.mark.parametrize("prec", [BF16, BF16M], ids=["bf16", "bf16_mixed"])
def test_bf16_water_box(cfg2, prec):
    mc, s, w, sc, sh, ref = cfg2
    m = gpu_model(mc, w, prec, sc, sh)
    got = gpu_eval(m, s)
    _check_bf16(f"cfg2_{'bf16' if prec == BF16 else 'bf16_mixed'}", got, ref, s.n_local)


def test_bf16_single_rounded_weights_forces(cfg2):
    """Single-rounded BF16 weights: forces stay within 1 % RMS; the energy
    carries the systematic weight-rounding error (reported, not gated)."""
    mc, s, w, sc, sh, ref = cfg2
    got = gpu_eval(gpu_model(mc, w, BF16S, sc, sh), s)
    dE = abs(float(got["energy"][0]) - ref.energy) / s.n_local
    rel = float(np.sqrt(((got["forces"] - ref.forces) ** 2).mean()) / np.sqrt((ref.forces ** 2).mean()))
    _report("cfg2_bf16_single", dE_per_atom=dE, force_rel_rms=rel)
    assert rel <= 0.01


def test_chunked_equals_whole(cfg2):
    mc, s, w, sc, sh, ref = cfg2
    a = gpu_eval(gpu_model(mc, w, FP32, sc, sh), s)
    b = gpu_eval(gpu_model(mc, w, FP32, sc, sh, edge_chunk=9000), s)
    assert np.array_equal(a["forces"], b["forces"])
    assert np.array_equal(a["atom_energy"], b["atom_energy"])


def test_bf16_tile_shapes_agree(cfg2):
    """The 128-, 64- and 32-edge BF16 MLP kernels compute the same products in
    the same K order: energies agree exactly; forces agree to the level of one
    BF16 rounding of an activation (the kernels' compiled float expressions may
    round an intermediate differently before it is rounded to BF16)."""
    mc, s, w, sc, sh, ref = cfg2
    outs = {t: gpu_eval(gpu_model(mc, w, BF16, sc, sh, mlp_tile=t), s) for t in (128, 64, 32)}
    fs = float(np.sqrt((outs[64]["forces"] ** 2).mean()))
    for t in (128, 32):
        d = outs[t]["forces"] - outs[64]["forces"]
        rel_rms = float(np.sqrt((d ** 2).mean())) / fs
        _report(f"tiles_{t}_vs_64", max_dF=float(np.abs(d).max()), rel_rms=rel_rms,
                dE=float(outs[t]["energy"][0] - outs[64]["energy"][0]))
        assert np.array_equal(outs[t]["energy"], outs[64]["energy"])
        assert np.array_equal(outs[t]["atom_energy"], outs[64]["atom_energy"])
        assert rel_rms <= 2e-4


# Register-resident BF16 chains (256) against the LDS-staged ones, alone and
# mixed per kernel kind (they share the workspace conventions: the stored
# final-layer scalars, the staged dE/dx_out rows).
RR_TILES = [("rr_all", [256] * 6 + [32, 32]),
            ("rr_fwd_lds_bwd", [256, 256, 256, 64, 64, 64, 32, 32]),
            ("lds_fwd_rr_bwd", [64, 64, 64, 256, 256, 256, 16, 16])]


@pytest.mark.parametrize("prec", [BF16, BF16M], ids=["bf16", "bf16_mixed"])
@pytest.mark.parametrize("case", RR_TILES, ids=lambda c: c[0])
def test_register_resident_chains_water_box(cfg2, prec, case):
    mc, s, w, sc, sh, ref = cfg2
    name, tiles = case
    m = gpu_model(mc, w, prec, sc, sh)
    m.set_tiles(tiles)
    got = gpu_eval(m, s)
    _check_bf16(f"cfg2_{name}_{'bf16' if prec == BF16 else 'bf16_mixed'}", got, ref, s.n_local)
    assert np.allclose(got["atom_virial"].reshape(-1, 3, 3).sum(0), got["virial"].reshape(3, 3), atol=1e-6)


def test_repeatable_bitwise(cfg2):
    mc, s, w, sc, sh, ref = cfg2
    m = gpu_model(mc, w, BF16, sc, sh)
    a, b = gpu_eval(m, s), gpu_eval(m, s)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


SMALL = [
    ("one_layer_lmax1", dict(l_max=1, n_layers=1, n_tensor=8, twobody_dims=(32, 32), latent_dims=(32, 32))),
    ("two_layer_lmax1_n16", dict(l_max=1, n_layers=2, n_tensor=16, twobody_dims=(64,), latent_dims=(64,))),
    ("no_channel_mix", dict(l_max=2, n_layers=2, n_tensor=32, twobody_dims=(64, 64), latent_dims=(64, 64),
                            channel_mix=False)),
    ("one_layer_lmax2_n64", dict(l_max=2, n_layers=1, n_tensor=64, twobody_dims=(128, 128, 128),
                                 latent_dims=(128, 128, 128))),
    ("uneven_widths", dict(l_max=2, n_layers=2, n_tensor=16, twobody_dims=(48, 96, 80), latent_dims=(112, 80))),
]


# (precision, MLP edge-tile rows): every tile shape of both precisions
PREC_TILES = [(FP32, 32), (FP32, 16), (BF16, 128), (BF16, 64), (BF16, 32), (BF16M, 128), (BF16M, 64)]
_PNAME = {FP32: "fp32", BF16: "bf16", BF16M: "bf16mixed"}


@pytest.mark.parametrize("case", SMALL, ids=lambda c: c[0])
@pytest.mark.parametrize("prec,tile", PREC_TILES, ids=[f"{_PNAME[p]}_tile{t}" for p, t in PREC_TILES])
def test_small_models(case, prec, tile):
    name, kw = case
    mc = W.ModelConfig(n_species=2, r_cut=4.0, **kw)
    w = W.make_weights(mc, np.random.default_rng(5))
    s = W.system(1)
    sc, sh = W.species_scale_shift(mc, np.random.default_rng(6))
    ref = OM.evaluate(mc, w, s, sc, sh)
    got = gpu_eval(gpu_model(mc, w, prec, sc, sh, mlp_tile=tile), s)
    if prec == FP32:
        _check_fp32(name, got, ref, s.n_local)
    else:
        _check_bf16(name, got, ref, s.n_local)


def test_clusters_and_ghost_shell_fp32():
    mc = W.model_config(4)
    w = W.make_weights(mc, np.random.default_rng(8))
    cl = W.clusters(5, 3, lo=20, hi=300)
    ref = OM.evaluate(mc, w, cl)
    got = gpu_eval(gpu_model(mc, w, FP32), cl)
    _check_fp32("clusters", got, ref, cl.n_local)
    # ghost-shell share of a periodic box = the periodic box
    s = W.jittered_lattice_box(1000, (1000 / 0.1) ** (1 / 3), 0.5, W.PROTEIN_MIX, 12)
    g = W.ghost_shell(s, 6.0)
    m = gpu_model(mc, w, FP32)
    a, b = gpu_eval(m, s), gpu_eval(m, g)
    F = b["forces"][:s.n_local].copy()
    np.add.at(F, g.ghost_owner, b["forces"][s.n_local:])
    # identical up to FP32 summation order (neighbour order differs)
    assert np.abs(a["atom_energy"] - b["atom_energy"]).max() < 1e-5
    assert np.abs(F - a["forces"]).max() < 1e-4


def test_empty_and_isolated():
    mc = W.model_config(2)
    w = W.make_weights(mc, np.random.default_rng(1))
    sc, sh = W.species_scale_shift(mc, np.random.default_rng(2))
    s = W.System(pos=np.array([[0.0, 0.0, 0.0], [10.0, 0.0, 0.0]]), species=np.array([0, 1], np.int32),
                 cell=np.zeros(3), pbc=np.zeros(3, np.int32), n_local=2)
    got = gpu_eval(gpu_model(mc, w, BF16, sc, sh), s)
    assert np.all(got["forces"] == 0.0)
    assert np.allclose(got["atom_energy"], sh[[0, 1]])
    s0 = W.System(pos=np.zeros((0, 3)), species=np.zeros(0, np.int32), cell=np.zeros(3),
                  pbc=np.zeros(3, np.int32), n_local=0)
    got = gpu_eval(gpu_model(mc, w, BF16, sc, sh), s0)
    assert got["energy"][0] == 0.0


# The full-size protein box (whole-box fixture, every tile shape) is covered
# by test_gpu_protein_box.py.


# ----------------------------------------------------------------------------- interface behaviour

def test_error_paths():
    mc = W.model_config(2)
    w = W.make_weights(mc, np.random.default_rng(1))
    m = gpu_model(mc, w, BF16)
    s = W.system(1)
    pos, sp = to_dev(s)
    F = torch.empty((s.n_total, 3), dtype=torch.float64, device=pos.device)
    with pytest.raises(P.AllegroError) as ex:
        m.energy_forces(pos, sp, F)
    assert ex.value.status == -6
    bad = pos.clone()
    bad[3, 1] = float("nan")
    with pytest.raises(P.AllegroError) as ex:
        m.neighbors(bad, sp, s.cell, s.pbc)
    assert ex.value.status == -5
    with pytest.raises(P.AllegroError) as ex:
        m.neighbors(pos, sp, [8.6, 0.1, 0, 0, 8.6, 0, 0, 0, 8.6], s.pbc)
    assert ex.value.status == -1
    for bad_tiles in ([16] * 6 + [0, 0], [0] * 6 + [64, 0]):   # 16-row MLP tiles are FP32-only
        with pytest.raises(P.AllegroError) as ex:
            m.set_tiles(bad_tiles)
        assert ex.value.status == -1
    # the model stays usable after errors
    got = gpu_eval(m, s)
    assert np.isfinite(got["energy"][0])


def test_nonfinite_outputs_reported():
    """Two atoms at the same position: the pair direction (and the radial
    basis sin(k d)/d) is undefined, the kernels produce NaN without faulting,
    and allegro_check reports ALLEGRO_E_NONFINITE; the record is then cleared
    and the model stays usable."""
    mc = W.model_config(2)
    w = W.make_weights(mc, np.random.default_rng(1))
    m = gpu_model(mc, w, FP32)
    pos = np.array([[0.0, 0.0, 0.0], [1.2, 0.3, 0.1], [1.2, 0.3, 0.1], [2.5, 0.0, 0.0]])
    s = W.System(pos=pos, species=np.array([1, 0, 0, 1], np.int32), cell=np.zeros(3),
                 pbc=np.zeros(3, np.int32), n_local=4)
    with pytest.raises(P.AllegroError) as ex:
        gpu_eval(m, s)
    assert ex.value.status == -5
    m.check()                                  # cleared by the report
    ok = W.System(pos=pos[[0, 1, 3]], species=np.array([1, 0, 1], np.int32), cell=np.zeros(3),
                  pbc=np.zeros(3, np.int32), n_local=3)
    ref = OM.evaluate(mc, w, ok)
    got = gpu_eval(m, ok)
    _check_fp32("after_nonfinite", got, ref, 3)


@pytest.mark.parametrize("prec", [FP32, BF16M], ids=["fp32", "bf16_mixed"])
def test_autotune_water_box(cfg2, prec):
    """allegro_autotune picks per-kernel tile shapes; the evaluation at those
    shapes matches the oracle."""
    mc, s, w, sc, sh, ref = cfg2
    m = gpu_model(mc, w, prec, sc, sh)
    pos, sp = to_dev(s)
    m.neighbors(pos, sp, s.cell, s.pbc, s.n_local)
    picks = m.autotune(pos, sp)
    _report(f"cfg2_autotune_{_PNAME[prec]}", **{k: int(v) for k, v in picks.items()})
    got = gpu_eval(m, s)
    if prec == FP32:
        _check_fp32("cfg2_autotuned", got, ref, s.n_local)
    else:
        _check_bf16("cfg2_autotuned", got, ref, s.n_local)


def test_autograd_function():
    from paper_2304_10061_amd.autograd import energy
    mc, s, w = W.workload(1)
    m = gpu_model(mc, w, FP32)
    pos, sp = to_dev(s)
    pos.requires_grad_(True)
    E = energy(pos, m, sp, s.cell, s.pbc)
    E.backward()
    ref = OM.evaluate(mc, w, s)
    assert abs(E.item() - ref.energy) / s.n_local < 1e-6
    assert np.abs(-pos.grad.cpu().numpy() - ref.forces).max() < 1e-4
