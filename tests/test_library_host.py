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
