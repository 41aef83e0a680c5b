"""CPU checks of the C interface: the library loads, exports every declared
symbol, and its host-side logic (configuration validation, weight count, path
enumeration) agrees with the oracle's independent enumeration.  No GPU work."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2304_10061_amd as P
from paper_2304_10061_amd import binding
import workloads as W
from oracle import cg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "allegro_mi355x.h")).read()
    return sorted(set(re.findall(r"\b(allegro_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = P.load_library()
    decl = _declared()
    assert len(decl) >= 10
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTS) == decl


def _check_describe(mc):
    info = P.describe(P.config_from(mc))
    paths = cg.layer_paths(mc.l_max, mc.n_layers)
    widths = cg.layer_widths(mc.l_max, mc.n_layers)
    assert [info.n_paths[k] for k in range(mc.n_layers)] == [len(p) for p in paths]
    rng = np.random.default_rng(0)
    lm1 = mc.l_max + 1
    shape = (2, lm1, lm1, lm1) if cg.has_unnatural(mc.l_max, mc.n_layers) else (lm1, lm1, lm1)
    nnz = [np.count_nonzero(cg.fused_table(mc.l_max, p, rng.standard_normal(shape), k == len(paths) - 1,
                                           *widths[k]))
           for k, p in enumerate(paths)]
    assert [info.n_nonzero[k] for k in range(mc.n_layers)] == nnz
    assert [info.width[k] for k in range(mc.n_layers)] == [w[1] for w in widths]
    assert info.n_weights == W.pack_weights(mc, W.make_weights(mc, rng)).size
    assert info.dim == (mc.l_max + 1) ** 2 and info.latent == mc.latent


@pytest.mark.parametrize("cfg", [1, 2, 3, 4])
def test_describe_matches_oracle(cfg):
    _check_describe(W.model_config(cfg))


@pytest.mark.parametrize("l_max,n_layers", [(1, 3), (2, 3), (3, 3), (3, 2), (3, 1), (1, 4), (2, 4), (3, 4)])
def test_describe_matches_oracle_deep(l_max, n_layers):
    """Deeper models carry unnatural-parity irreps: the library's pattern kinds
    must reproduce the oracle's pruned path sets, table non-zeros and widths."""
    _check_describe(W.ModelConfig(n_species=2, r_cut=4.0, l_max=l_max, n_layers=n_layers, n_tensor=32,
                                  twobody_dims=(64, 64), latent_dims=(64, 64), edge_dims=(32,)))


@pytest.mark.parametrize("bad", [dict(l_max=4), dict(n_layers=5), dict(l_max=3, n_tensor=16),
                                 dict(n_layers=3, n_tensor=8), dict(l_max=3, n_bessel=12),
                                 dict(n_tensor=24), dict(n_species=20),
                                 dict(twobody_dims=(100, 100), latent_dims=(100, 100)),
                                 dict(latent_dims=(64, 32)), dict(edge_dims=(64, 64)), dict(r_cut=-1.0),
                                 dict(r_cut_pair=((3.0, 4.5), (3.0, 4.0))),      # above r_cut
                                 dict(r_cut_pair=((3.0, 0.0), (3.0, 4.0))),      # not positive
                                 dict(r_cut_pair=((3.0, float("nan")), (3.0, 4.0))),
                                 dict(atomic_numbers=(0, 8)), dict(atomic_numbers=(1, 119))])
def test_describe_rejects_unsupported(bad):
    kw = dict(n_species=2, r_cut=4.0, l_max=2, n_layers=2, n_tensor=32, twobody_dims=(64, 64),
              latent_dims=(64, 64), edge_dims=(32,))
    kw.update(bad)
    with pytest.raises(P.AllegroError) as ex:
        P.describe(P.make_config(**kw))
    assert ex.value.status == -1


def test_create_rejects_wrong_weight_count_without_device_work():
    mc = W.model_config(2)
    cfg = P.config_from(mc)
    lib = P.load_library()
    w = np.zeros(10, np.float32)
    h = ctypes.c_void_p()
    st = lib.allegro_create(ctypes.byref(cfg), w.ctypes.data, w.size, None, None, ctypes.byref(h))
    assert st == -1 and not h.value
    assert b"n_weights" in lib.allegro_last_error(None)
    assert lib.allegro_status_string(-3) == b"ALLEGRO_E_CAPACITY"
    assert lib.allegro_num_edges(None) == -1
    lib.allegro_destroy(None)


def test_describe_accepts_pair_cutoffs():
    kw = dict(n_species=2, r_cut=4.0, l_max=2, n_layers=2, n_tensor=32, twobody_dims=(64, 64),
              latent_dims=(64, 64), edge_dims=(32,))
    a = P.describe(P.make_config(**kw))
    b = P.describe(P.make_config(r_cut_pair=W.paper_pair_cutoffs(2, 4.0), **kw))
    assert a.n_weights == b.n_weights
    with pytest.raises(ValueError):
        P.make_config(r_cut_pair=((3.0, 4.0),), **kw)


# ----------------------------------------------------------------------------- 32-bit workspace offsets

def _deep4_lmax3_n64():
    return W.ModelConfig(n_species=2, r_cut=4.0, l_max=3, n_layers=4, n_tensor=64,
                         twobody_dims=(128, 128), latent_dims=(128, 128), edge_dims=(128,))


@pytest.mark.parametrize("name,mc,widest", [
    ("protein_box_model", W.model_config(3), 9 * 64),            # V of the first layer: dim n floats per edge
    ("subdomain_model", W.model_config(4), 3 * 3 * 32),          # [a0 | w^1] head: 2 (l_max+1) n = dim n
    ("deep4_lmax3_n64", _deep4_lmax3_n64(), 2 * 16 * 64),        # both-parity features: 2 dim n
])
def test_chunk_cap_keeps_offsets_below_2_31(name, mc, widest):
    info = P.describe(P.config_from(mc))
    assert info.widest_row == widest
    assert info.max_chunk_edges > 0
    assert info.max_chunk_edges * info.widest_row < 2 ** 31
    assert (info.max_chunk_edges + 1) * info.widest_row >= 2 ** 31 - 1


def _check_plan(bounds, counts, cap):
    assert bounds[0] == 0 and bounds[-1] == len(counts)
    assert np.all(np.diff(bounds) > 0)
    rp = np.concatenate([[0], np.cumsum(counts, dtype=np.int64)])
    per = rp[bounds[1:]] - rp[bounds[:-1]]
    assert per.max() <= cap
    # greedy: no chunk could have taken the next centre as well
    nxt = rp[np.minimum(bounds[1:-1] + 1, len(counts))] - rp[bounds[:-2]]
    assert np.all(nxt > cap)
    return per


def test_plan_chunks_one_gpu_subdomain_share():
    """The 1M-atom subdomain with its ghost shell: about 27 neighbours per
    centre, ~32M edges, more than one chunk may hold at 288 floats per edge
    row -- the list is split into whole-centre chunks automatically."""
    mc = W.model_config(4)
    rng = np.random.default_rng(0)
    counts = rng.poisson(31.7, size=1_000_000).astype(np.int32)
    cfg = P.config_from(mc, edge_chunk=0)
    info = P.describe(cfg)
    b = P.plan_chunks(cfg, counts)
    per = _check_plan(b, counts, info.max_chunk_edges)
    assert len(b) - 1 >= int(np.ceil(counts.sum() / info.max_chunk_edges))
    assert per.max() * info.widest_row < 2 ** 31
    # an explicit bound below the cap is kept, one above it is reduced
    small = P.plan_chunks(P.config_from(mc, edge_chunk=4_000_000), counts)
    _check_plan(small, counts, 4_000_000)
    big = P.plan_chunks(P.config_from(mc, edge_chunk=10 ** 12), counts)
    assert np.array_equal(big, b)


def test_plan_chunks_deep_model_and_limits():
    mc = _deep4_lmax3_n64()
    cfg = P.config_from(mc)
    info = P.describe(cfg)
    counts = np.full(400_000, 60, np.int32)            # 24M edges at 2048 floats per row
    b = P.plan_chunks(cfg, counts)
    per = _check_plan(b, counts, info.max_chunk_edges)
    assert per.max() * info.widest_row < 2 ** 31
    # a centre with more neighbours than a chunk may hold is rejected
    bad = counts.copy()
    bad[7] = info.max_chunk_edges + 1
    with pytest.raises(P.AllegroError) as ex:
        P.plan_chunks(cfg, bad)
    assert ex.value.status == -1
    # empty input: a single boundary
    assert list(P.plan_chunks(cfg, np.zeros(0, np.int32))) == [0]


def test_noalloc_scratch_size_matches_header():
    """The binding's copy of the static workspace size equals the header's."""
    txt = open(os.path.join(ROOT, "include", "allegro_mi355x.h")).read()
    m = re.search(r"#define ALLEGRO_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", txt)
    assert m is not None
    assert int(m.group(1)) << int(m.group(2)) == binding.NOALLOC_SCRATCH_BYTES
