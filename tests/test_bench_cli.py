"""bench.py refuses multi-GPU runs (it measures one GPU's share)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_rejects_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_mac_counts():
    sys.path.insert(0, ROOT)
    import bench
    import workloads as W
    macs = bench.mlp_macs_per_edge(W.model_config(3))
    # two-body chain 16->256->256->256 plus the [embed0 | env1] head 256 -> 384
    assert macs["mlp_fwd_twobody"] == 16 * 256 + 2 * 256 * 256 + 256 * 384
    # latent chain (256+64)->256->256->256 plus the env2 head 256 -> 192
    assert macs["mlp_fwd_latent"] == 320 * 256 + 2 * 256 * 256 + 256 * 192
    assert macs["mlp_bwd_final"] == 320 * 256 + 2 * 256 * 256


def test_tensor_flop_counts():
    """Tensor-track flops per edge of the two-layer water model, by hand:
    n = 32, 9 components, 83 / 9 table non-zeros."""
    sys.path.insert(0, ROOT)
    import bench
    import paper_2304_10061_amd as P
    import workloads as W
    mc = W.model_config(2)
    f = bench.tensor_flops_per_edge(mc, P.describe(P.config_from(mc)))
    assert f["env"] == 2 * 2 * 9 * 32
    assert f["tp_mix"] == 2 * 83 * 32 + 2 * 32 * 32 * 9
    assert f["mix_adjoint"] == 3 * 9 * 32 + 2 * 32 * 32 * 9
    assert f["tp_env_adjoint"] == 2 * (2 * 83 * 32 + 4 * 9 * 32)
    assert f["tp_env_adjoint_final"] == 2 * 9 * 32 + 4 * 9 * 32


def test_tensor_unit_bytes():
    """Algorithmic bytes per edge of the tensor-track units on the protein
    box (l_max 2, n 64): a staged non-final tensor product moves one 9 x 64
    FP32 row in and one out (4,608 B, the ~4.6 KB of the staged estimate),
    an environment scatter the 3 x 64 weights and 9 harmonics (804 B, ~0.8
    KB); the tensor adjoint unit is one of each."""
    sys.path.insert(0, ROOT)
    import bench
    import workloads as W
    b = bench.tensor_bytes_per_unit(W.model_config(3))
    assert b["tp_mix"] == 4 * 2 * 9 * 64 == 4608
    assert b["env"] == 4 * (3 * 64 + 9) == 804
    assert b["tp_env_adjoint"] == 4608 + 804
    assert b["tp_env_adjoint_final"] == 4 * 9 * 64 + 804


def test_tensor_symbols_name_profiled_kernels():
    """The kernel symbols the deep roofline sums are the ones the committed
    kernel-trace summary of that workload lists."""
    sys.path.insert(0, ROOT)
    import bench
    import workloads as W
    txt = open(os.path.join(ROOT, "profiles", "hbm_traffic_deep_water_box.md")).read()
    syms = bench.tensor_symbols(W.deep_model_config())
    for kind, names in syms.items():
        for s in names:
            assert s in txt, (kind, s)
    assert len(syms["tp_env_adjoint"]) == 4 and len(syms["tp_mix"]) == 2
