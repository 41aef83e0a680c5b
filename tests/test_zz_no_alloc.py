"""allegro_energy_forces_noalloc (the entry point for callers that cannot
allocate) against allegro_energy_forces on the same neighbour list: the same
kernels on the library's static per-GPU workspace, so every output must be
identical.  Two calls in a row, the second on a smaller input (the static
workspace then holds the first call's contents), and the size check."""
import numpy as np
import pytest
import torch

import paper_2304_10061_amd as P
import workloads as W

from gpu_helpers import to_dev

pytestmark = pytest.mark.gpu


def _eval(model, s, fn):
    pos, sp = to_dev(s)
    dev = pos.device
    n_total, n_local = s.pos.shape[0], s.n_local
    out = {"forces": torch.empty((n_total, 3), dtype=torch.float64, device=dev),
           "atom_energy": torch.empty(n_local, dtype=torch.float64, device=dev),
           "virial": torch.empty(9, dtype=torch.float64, device=dev),
           "atom_virial": torch.empty((n_total, 9), dtype=torch.float64, device=dev),
           "energy": torch.empty(1, dtype=torch.float64, device=dev)}
    fn(pos, sp, out["forces"], out["atom_energy"], out["virial"], out["atom_virial"], out["energy"])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("prec", [P.PREC_FP32, P.PREC_BF16_MIXED], ids=["fp32", "bf16_mixed"])
def test_noalloc_equals_allocating_entry_point(prec):
    mc = W.model_config(2)
    w = W.make_weights(mc, W.seeds(2)[3])
    # the 3,000-atom water box (about 80k edges) in chunks of at most 20k
    # edges, then a 700-atom box: the second call is smaller than the first
    big = W.jittered_lattice_box(3000, 31.1, 0.4, W.WATER_MIX, 11)
    small = W.jittered_lattice_box(700, (700 / 0.1) ** (1 / 3), 0.4, W.WATER_MIX, 12)
    m = P.Model(P.config_from(mc, precision=prec, edge_chunk=20000), W.pack_weights(mc, w))
    for tag, s in (("water3000", big), ("water700", small)):
        pos, sp = to_dev(s)
        m.neighbors(pos, sp, s.cell, s.pbc, s.n_local)
        ref = _eval(m, s, m.energy_forces)
        got = _eval(m, s, m.energy_forces_noalloc)
        print(tag, "edges", m.num_edges(), "E", float(got["energy"][0]), flush=True)
        for k in ref:
            assert np.array_equal(got[k], ref[k]), (tag, k)


def test_noalloc_rejects_a_list_beyond_its_workspace():
    mc = W.model_config(2)
    w = W.make_weights(mc, W.seeds(2)[3])
    s = W.jittered_lattice_box(3000, 31.1, 0.4, W.WATER_MIX, 11)
    m = P.Model(P.config_from(mc, precision=P.PREC_FP32), W.pack_weights(mc, w))   # one chunk of ~80k edges
    pos, sp = to_dev(s)
    m.neighbors(pos, sp, s.cell, s.pbc, s.n_local)
    forces = torch.empty((s.pos.shape[0], 3), dtype=torch.float64, device=pos.device)
    with pytest.raises(P.AllegroError) as ei:
        m.energy_forces_noalloc(pos, sp, forces)
    assert ei.value.status == -1 and "edge_chunk" in str(ei.value)
