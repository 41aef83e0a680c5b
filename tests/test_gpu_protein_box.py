"""Whole-box parity of the 23,558-atom protein-like box (the benchmark
workload, 2.05M ordered edges) against the FP64 oracle, at every edge-tile
shape the benchmark can run.

The reference is tests/golden/protein_box_reference.npz, written by
tests/golden/make_protein_box_reference.py, which calls only `oracle/`
(energy, virial, all 23,558 atom energies and all 70,674 force components).

Gates (FP64 oracle as reference):
  FP32         |E - E_ref| / N <= 1e-6 eV/atom, max |F - F_ref| <= 1e-4 eV/A
  BF16 modes   |E - E_ref| / N <= 1e-3 eV/atom, RMS(F - F_ref) <= 1% of RMS(F_ref)
"""
import os

import numpy as np
import pytest
import torch

import paper_2304_10061_amd as P
import workloads as W

from gpu_helpers import gpu_eval, gpu_model, to_dev

pytestmark = pytest.mark.gpu

FP32, BF16, BF16M = P.PREC_FP32, P.PREC_BF16, P.PREC_BF16_MIXED
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "protein_box_reference.npz")

# Tile sets, in the order mlp_fwd_twobody, mlp_fwd_latent, mlp_fwd_final,
# mlp_bwd_final, mlp_bwd_latent, mlp_bwd_twobody, tp_mix, mix_adjoint.
# Together they run every kernel instantiation the benchmark's autotuner can
# pick at d = 256, n = 64: the register-resident BF16 chains (256), 128-row
# (two column tiles per wave), 64- and 32-row MLP tiles in BF16, 32- and
# 16-row in FP32, and 32- and 16-edge tensor-product / mixing tiles.
CASES = [
    ("fp32_rows32_tp32", FP32, [32] * 6 + [32, 32]),
    ("fp32_rows16_tp16", FP32, [16] * 6 + [16, 16]),
    ("bf16mixed_default", BF16M, None),
    ("bf16mixed_rr_tp16", BF16M, [256] * 6 + [16, 16]),
    ("bf16mixed_rr_tp32", BF16M, [256] * 6 + [32, 32]),
    ("bf16_pairs_rr_tp16", BF16, [256] * 6 + [16, 16]),
    ("bf16mixed_rr_fwd_lds_bwd", BF16M, [256, 256, 256, 64, 64, 64, 16, 16]),
    ("bf16mixed_lds_fwd_rr_bwd", BF16M, [128, 128, 32, 256, 256, 256, 16, 16]),
    ("bf16mixed_rows128_tp16", BF16M, [128] * 6 + [16, 16]),
    ("bf16mixed_rows64_tp32", BF16M, [64] * 6 + [32, 32]),
    ("bf16mixed_rows32_tp16", BF16M, [32] * 6 + [16, 16]),
    ("bf16mixed_bench_pick", BF16M, [128, 128, 32, 64, 64, 64, 16, 16]),
    ("bf16_pairs_rows128_tp16", BF16, [128] * 6 + [16, 16]),
]


def _report(tag, **kw):
    print(tag, " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.fixture(scope="module")
def box():
    ref = np.load(GOLDEN, allow_pickle=False)
    mc, s, w = W.workload(3)
    return mc, s, w, ref


def _gate(tag, prec, got, ref, n):
    F_ref = ref["forces"].astype(np.float64)
    dF = got["forces"] - F_ref
    dE = abs(float(got["energy"][0]) - float(ref["energy"])) / n
    dEi = np.abs(got["atom_energy"] - ref["atom_energy"].astype(np.float64))
    frms = float(np.sqrt((F_ref ** 2).mean()))
    rel = float(np.sqrt((dF ** 2).mean())) / frms
    dW = float(np.abs(got["virial"].reshape(3, 3) - ref["virial"]).max())
    _report(tag, dE_per_atom=dE, max_dEi=float(dEi.max()), max_dF=float(np.abs(dF).max()), force_rel_rms=rel,
            max_dW=dW, Frms=frms)
    if prec == FP32:
        assert dE <= 1e-6
        assert float(np.abs(dF).max()) <= 1e-4
        assert dW <= 1e-4 * max(1.0, float(np.abs(ref["virial"]).max()))
    else:
        assert dE <= 1e-3
        assert rel <= 0.01
    # periodic box: zero net force up to FP32 accumulation
    assert np.abs(got["forces"].sum(0)).max() < 1e-6 * n


@pytest.mark.parametrize("case", CASES, ids=lambda c: c[0])
def test_protein_box_whole(box, case):
    name, prec, tiles = case
    mc, s, w, ref = box
    m = gpu_model(mc, w, prec)
    if tiles is not None:
        m.set_tiles(tiles)
    got = gpu_eval(m, s, want_atom_virial=False)
    assert m.num_edges() == int(ref["n_edges"])
    _gate(f"cfg3_{name}", prec, got, ref, s.n_local)


@pytest.mark.parametrize("prec", [FP32, BF16M], ids=["fp32", "bf16_mixed"])
def test_protein_box_autotuned(box, prec):
    """allegro_autotune on the benchmark box, then the whole box at the
    shapes it chose."""
    mc, s, w, ref = box
    m = gpu_model(mc, w, prec)
    pos, sp = to_dev(s)
    m.neighbors(pos, sp, s.cell, s.pbc, s.n_local)
    picks = m.autotune(pos, sp)
    torch.cuda.synchronize()
    _report(f"cfg3_autotune_{'fp32' if prec == FP32 else 'bf16mixed'}", **{k: int(v) for k, v in picks.items()})
    allowed_mlp = {32, 16} if prec == FP32 else {256, 128, 64, 32}
    assert all(picks[k] in allowed_mlp for k in P.Model.TILE_KINDS[:6])
    assert all(picks[k] in (16, 32) for k in P.Model.TILE_KINDS[6:])
    got = gpu_eval(m, s, want_atom_virial=False)   # keeps the tuned shapes
    _gate("cfg3_autotuned", prec, got, ref, s.n_local)
