"""Per-ordered-species-pair cutoffs (section "Species-dependent cutoffs") on
the HIP path, against the FP64 oracle: neighbour lists bit-exact, FP32 and
BF16-mixed energies and forces at the tolerances of the other parity tests,
and a neighbour skin that adds only pairs with a zero envelope.  Cutoffs: the
paper's H-H 3.0, H-C 1.25, H-O 1.25, O-H 3.0 A, every other ordered pair the
model's r_c.
"""
import copy

import numpy as np
import pytest

import paper_2304_10061_amd as P
import workloads as W
from oracle import model as OM
from oracle.neighbors import neighbor_list

from gpu_helpers import gpu_edges, gpu_eval, gpu_model
from test_gpu_parity import _check_bf16, _check_fp32, _report

pytestmark = pytest.mark.gpu


def with_pairs(mc):
    m = copy.copy(mc)
    m.pair_cutoffs = W.paper_pair_cutoffs(mc.n_species, mc.r_cut)
    return m


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_pair_cutoff_neighbors_bit_exact(cfg):
    mc = with_pairs(W.model_config(cfg))
    s = W.system(cfg)
    m = gpu_model(mc, W.make_weights(mc, np.random.default_rng(0)), P.PREC_FP32)
    i, j, sh = gpu_edges(m, s)
    ri, rj, rs = neighbor_list(s.pos, s.cell, s.pbc, mc.r_cut, n_local=s.n_local, species=s.species,
                               pair_cutoffs=mc.pair_cutoffs, method="kdtree" if cfg == 3 else "auto")
    full = len(neighbor_list(s.pos, s.cell, s.pbc, mc.r_cut, n_local=s.n_local,
                             method="kdtree" if cfg == 3 else "auto")[0])
    _report(f"cfg{cfg}_pairs", edges=len(ri), single_cutoff_edges=full, ratio=full / max(len(ri), 1))
    assert np.array_equal(i, ri) and np.array_equal(j, rj) and np.array_equal(sh, rs)
    assert len(ri) < full


@pytest.fixture(scope="module")
def water_pairs():
    mc, s, w = W.workload(2)
    mc = with_pairs(mc)
    sc, sh = W.species_scale_shift(mc, np.random.default_rng(21))
    ref = OM.evaluate(mc, w, s, sc, sh)
    return mc, s, w, sc, sh, ref


def test_pair_cutoff_fp32_water_box(water_pairs):
    mc, s, w, sc, sh, ref = water_pairs
    got = gpu_eval(gpu_model(mc, w, P.PREC_FP32, sc, sh), s)
    _check_fp32("cfg2_pairs_fp32", got, ref, s.n_local)


def test_pair_cutoff_bf16_mixed_water_box(water_pairs):
    mc, s, w, sc, sh, ref = water_pairs
    got = gpu_eval(gpu_model(mc, w, P.PREC_BF16_MIXED, sc, sh), s)
    _check_bf16("cfg2_pairs_bf16_mixed", got, ref, s.n_local)


def test_pair_cutoff_skin_adds_only_zero_pairs(water_pairs):
    mc, s, w, sc, sh, ref = water_pairs
    a = gpu_eval(gpu_model(mc, w, P.PREC_FP32, sc, sh), s)
    cfg = P.config_from(mc, precision=P.PREC_FP32, neighbor_skin=0.6)
    m = P.Model(cfg, W.pack_weights(mc, w), sc, sh)
    b = gpu_eval(m, s)
    n_skin = m.num_edges()
    _report("cfg2_pairs_skin", edges_with_skin=n_skin, edges=len(ref.edge_energy))
    assert n_skin > len(ref.edge_energy)
    assert abs(float(a["energy"][0]) - float(b["energy"][0])) / s.n_local <= 1e-7
    assert float(np.abs(a["forces"] - b["forces"]).max()) <= 1e-5
