#!/usr/bin/env python3
"""Throughput of the Allegro energy+force path on one MI355X.

One step = allegro_neighbors + allegro_energy_forces (energy, per-atom
energies, forces, virial) on the 23,558-atom protein-like periodic box
(0.1 atoms/A^3, H:C:N:O = 50:30:8:12, r_c = 6 A; model: 8 Bessel, l_max 2,
2 layers, 64 tensor channels, latent MLPs [256, 256, 256], edge MLP [128]),
seeded synthetic positions and weights already resident in HBM.

The headline value is BF16-mixed atom-steps/s (MLP GEMMs in BF16 on MFMA with
FP32 accumulation); the plain FP32 path on the same GPU is reported beside it.
`roofline` describes the dominant kernel, timed with HIP events on the stream
it runs on; `cpu_baseline` is the FP64 oracle on the host cores on a bounded
sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import copy
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BF16_PEAK_TFLOPS = 2500.0     # MI355X dense BF16 MFMA
FP32_PEAK_TFLOPS = 157.3      # MI355X dense FP32 MFMA
HBM_PEAK_GBS = 8000.0         # MI355X HBM3E

# Kernel symbol (as rocprofv3 prints it) of each timed MLP launch kind, for
# precision p: template arguments <precision, kind, tile rows, column tiles>.
MLP_KIND = {"twobody": 0, "latent": 1, "final": 2}
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hbm_traffic_protein_box.md")
TRAFFIC_SUMMARY_DEEP = os.path.join(ROOT, "profiles", "hbm_traffic_deep_water_box.md")


MLP_WAVES = 8                 # waves per MLP block
TALL_ROWS = 128               # tile rows of the in-place (tall) MLP kernels
RR_TILE = 256                 # tile code of the register-resident MLP kernels
SIMDS = 1024                  # 256 CUs x 4 SIMDs
CLOCK_GHZ = 2.4               # peak engine clock (the clock of the MFMA peak)


def mlp_symbol(launch, precision, tile_rows, latent):
    """'mlp_bwd_final', 1, 32, 256 -> 'k_mlp_bwd<1, 2, 32, 2>' (the kernel's name
    without namespace and arguments; the last argument is the column tiles per
    wave, ceil(d / (16 * MLP_WAVES))); 128-row tiles -> 'k_mlp_bwd_t<1, 2, 2>';
    register-resident kernels -> 'k_rr_bwd_final<' / 'k_rr_fwd<1, ' (prefixes)."""
    _, fb, kind = launch.split("_", 2)
    if tile_rows == RR_TILE:
        return f"k_rr_{fb}_final<" if kind == "final" else f"k_rr_{fb}<{MLP_KIND[kind]}, "
    ct = -(-(-(-latent // 16)) // MLP_WAVES)
    if tile_rows == TALL_ROWS:
        return f"k_mlp_{fb}_t<{precision}, {MLP_KIND[kind]}, {ct}>"
    return f"k_mlp_{fb}<{precision}, {MLP_KIND[kind]}, {tile_rows}, {ct}>"


def calibration_copy(mib):
    """A plain device-to-device copy of `mib` MiB (three times): the reference
    for scaling the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    a = torch.ones(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


def summarize_profiles(stats_dir, fetch_dir, write_dir, bench_log, copy_mib, commands, mfma_dir=None):
    """Markdown summary of a --kernel-trace --stats run and two --pmc runs
    (FETCH_SIZE, WRITE_SIZE): per-kernel average duration and counter values
    per dispatch, the copy-kernel scale factors, and the source hash.  With
    `mfma_dir` (a --pmc run of SQ_VALU_MFMA_BUSY_CYCLES and
    SQ_INSTS_VALU_MFMA_MOPS_BF16), also each kernel's matrix-core busy
    fraction, busy cycles / (1024 SIMDs x duration x 2.4 GHz) with the busy
    cycles summed over the SIMDs, and its executed BF16 MFMA rate (MOPS x 512
    flops / duration)."""
    import csv
    import glob

    def one(pattern):
        f = glob.glob(os.path.join(pattern, "**", "*.csv"), recursive=True)
        return f

    stats = {}
    for f in one(stats_dir):
        if f.endswith("kernel_stats.csv"):
            for r in csv.DictReader(open(f)):
                stats[r["Name"]] = (int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6)

    def counters(d, name):
        per = {}
        for f in one(d):
            if f.endswith("counter_collection.csv"):
                for r in csv.DictReader(open(f)):
                    if r["Counter_Name"] == name:
                        per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return per

    fetch, write = counters(fetch_dir, "FETCH_SIZE"), counters(write_dir, "WRITE_SIZE")
    busy = counters(mfma_dir, "SQ_VALU_MFMA_BUSY_CYCLES") if mfma_dir else {}
    mops = counters(mfma_dir, "SQ_INSTS_VALU_MFMA_MOPS_BF16") if mfma_dir else {}
    copy_kib = float(copy_mib) * 1024
    cf = max((v for k, vs in fetch.items() if "copyBuffer" in k for v in vs), default=None)
    cw = max((v for k, vs in write.items() if "copyBuffer" in k for v in vs), default=None)
    src_hash = None
    for line in open(bench_log):
        if line.startswith("{"):
            src_hash = json.loads(line).get("source_hash")
    blob = {"source_hash": src_hash, "copy_MiB": copy_mib,
            "copy_fetch_KiB": cf, "copy_write_KiB": cw,
            "fetch_scale": copy_kib / cf if cf else None, "write_scale": copy_kib / cw if cw else None,
            "kernels": {}}
    title = "protein-like box (23,558 atoms, 2.05M edges), BF16 step"
    for line in open(bench_log):
        if line.startswith("{"):
            rec = json.loads(line)
            cfg = rec.get("config", {})
            title = f"{rec.get('metric', title)}: {cfg.get('atoms', '?')} atoms, {cfg.get('edges', '?')} edges"
    lines = [f"# rocprofv3 summary: {title}", ""]
    for c in commands:
        lines.append(f"    {c}")
    lines += ["", "| kernel | calls | avg us | total ms | FETCH KiB/dispatch | WRITE KiB/dispatch |"
              " MFMA busy | BF16 MFMA TFLOP/s |",
              "|---|---|---|---|---|---|---|---|"]
    mean = lambda v: sum(v) / len(v) if v else None
    for name, (calls, avg, tot) in sorted(stats.items(), key=lambda kv: -kv[1][2])[:28]:
        fa, wa = mean(fetch.get(name)), mean(write.get(name))
        ba, ma = mean(busy.get(name)), mean(mops.get(name))
        bfrac = ba / (SIMDS * avg * 1e-6 * CLOCK_GHZ * 1e9) if ba is not None else None
        tfl = ma * 512 / (avg * 1e-6) / 1e12 if ma is not None else None
        short = name.replace("allegro::", "").replace("(anonymous namespace)::", "")[:90]
        lines.append(f"| `{short}` | {calls} | {avg:.1f} | {tot:.3f} | "
                     f"{'' if fa is None else f'{fa:.0f}'} | {'' if wa is None else f'{wa:.0f}'} | "
                     f"{'' if bfrac is None or not ba else f'{bfrac:.3f}'} | {'' if not ma else f'{tfl:.0f}'} |")
        if fa is not None and wa is not None:
            blob["kernels"][short] = {"avg_us": avg, "fetch_KiB": fa, "write_KiB": wa}
            if ba is not None:
                blob["kernels"][short].update({"mfma_busy_cycles": ba, "mfma_mops_bf16": ma})
    if copy_mib:
        lines += ["", "Counter scale factors from the plain copy of %d MiB (bytes per counted byte):" % copy_mib]
    else:
        lines += ["", "Kernel trace only (no counter passes); sources of the profiled build:"]
    lines += ["", "```json", json.dumps(blob, indent=1), "```", ""]
    return "\n".join(lines)


def kernel_source_hash():
    """SHA-256 over the HIP sources and headers of the library."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2304_10061_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def _summary_kernels(summary):
    try:
        txt = open(summary).read()
        blob = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("source_hash") != kernel_source_hash():
        return None
    return blob.get("kernels", {})


def mfma_busy_counters(symbols, summary=None):
    """Counter-derived matrix-core figures of the kernels whose names contain
    one of `symbols`, from the committed summary (None when it lacks them or
    the sources changed): busy fraction over their summed durations and
    executed BF16 MFMA TFLOP/s."""
    ks = _summary_kernels(summary or TRAFFIC_SUMMARY)
    if not ks:
        return None
    busy = mops = us = 0.0
    found = 0
    for name, k in ks.items():
        if "mfma_busy_cycles" in k and any(s in name for s in symbols):
            busy += k["mfma_busy_cycles"]
            mops += k["mfma_mops_bf16"] or 0.0
            us += k["avg_us"]
            found += 1
    if not found or us <= 0:
        return None
    return {"busy_frac": busy / (SIMDS * us * 1e-6 * CLOCK_GHZ * 1e9),
            "executed_bf16_tflops": mops * 512 / (us * 1e-6) / 1e12, "kernels": found}


def traffic_per_launch(symbol, summary=None):
    """HBM bytes per launch of `symbol` from the committed counter summary,
    or None when it is missing or the sources changed since it was taken."""
    try:
        txt = open(summary or TRAFFIC_SUMMARY).read()
        blob = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("source_hash") != kernel_source_hash():
        return None
    for name, k in blob.get("kernels", {}).items():
        if symbol in name:
            return k["fetch_KiB"] * 1024 * blob["fetch_scale"] + k["write_KiB"] * 1024 * blob["write_scale"]
    return None


def mlp_macs_per_edge(mc):
    """Algorithmic multiply-adds per edge of each MLP kernel kind: forward
    GEMMs (incl. the fused head), and input-gradient GEMMs of the adjoint
    (the adjoint's recomputation of the forward chain is not counted)."""
    d, n, LW = mc.latent, mc.n_tensor, (mc.l_max + 1) * mc.n_tensor

    def chain(dims):
        return sum(a * b for a, b in zip(dims[:-1], dims[1:]))

    two = chain([2 * mc.n_species + mc.n_bessel] + list(mc.twobody_dims))
    lat = chain([d + n] + list(mc.latent_dims))
    out = {
        "mlp_fwd_twobody": two + d * 2 * LW,
        "mlp_fwd_latent": lat + d * LW,
        "mlp_fwd_final": lat + d,
        "mlp_bwd_final": lat,
        "mlp_bwd_latent": lat + LW * d,
        "mlp_bwd_twobody": two + 2 * LW * d,
    }
    if mc.n_layers == 1:
        out.pop("mlp_fwd_latent")
        out.pop("mlp_bwd_latent")
    return out


def mlp_bytes_per_edge(mc):
    """HBM bytes per edge that each MLP kernel kind of this design stages:
    every input row read once and every output row written once (FP32
    arrays; per-centre and per-species rows, which stay in cache, are not
    counted).  These are the staged design's own I/O, not the method's
    minimum traffic."""
    d, n, LW, f = mc.latent, mc.n_tensor, (mc.l_max + 1) * mc.n_tensor, 4
    dim = (mc.l_max + 1) ** 2
    edge_in = f * (mc.n_bessel + 3)                 # radial basis, u and the species pair of the edge record
    out = {
        "mlp_fwd_twobody": edge_in + f * (d + 2 * LW),
        "mlp_fwd_latent": f * (d + n + 1) + f * (d + LW),
        "mlp_fwd_final": f * (d + dim * n + 1) + f * (1 + n),
        "mlp_bwd_final": f * (d + n + 1) + f * (d + n + 1),
        "mlp_bwd_latent": f * (d + LW + d + n + 1) + f * (d + n + 1),
        "mlp_bwd_twobody": edge_in + f * (d + 2 * LW) + f * (mc.n_bessel + 1),
    }
    if mc.n_layers == 1:
        out.pop("mlp_fwd_latent")
        out.pop("mlp_bwd_latent")
    return out


def tensor_flops_per_edge(mc, info):
    """Algorithmic FP32 flops per edge of each tensor-track launch kind, summed
    over the layers that launch it (timings are summed the same way): the
    fused tables' non-zeros (one multiply-add per non-zero and channel), the
    channel mixing (n^2 multiply-adds per mixed component) and the
    environment products (one multiply-add per harmonic component and
    channel).  Index arithmetic and the recomputation-free adjoint's
    bookkeeping are not counted."""
    n, D, nl = mc.n_tensor, (mc.l_max + 1) ** 2, mc.n_layers
    nnz = [int(info.n_nonzero[k]) for k in range(nl)]
    wout = [int(info.width[k]) for k in range(nl)]
    mixed = [(wout[k] - (1 if wout[k] > D else 0)) if mc.channel_mix else 0 for k in range(nl)]
    out = {"env": nl * 2 * D * n,
           "tp_env_adjoint_final": 2 * nnz[-1] * n + 4 * D * n + (2 * nnz[-1] * n + 4 * D * n if nl == 1 else 0)}
    if nl > 1:
        out["tp_mix"] = sum(2 * nnz[k] * n + 2 * n * n * mixed[k] for k in range(nl - 1))
        out["mix_adjoint"] = sum((2 * nnz[k + 1] * n if k + 1 < nl - 1 else 3 * D * n) + 2 * n * n * mixed[k]
                                 for k in range(nl - 1))
        out["tp_env_adjoint"] = sum(2 * nnz[k] * n + 4 * D * n + (2 * nnz[k] * n + 4 * D * n if k == 0 else 0)
                                    for k in range(nl - 1))
    return out


def P_describe(mc):
    """allegro_describe of the model configuration (None without the library)."""
    try:
        import paper_2304_10061_amd as P
        return P.describe(P.config_from(mc))
    except Exception:
        return None


def tensor_bytes_per_unit(mc):
    """Algorithmic HBM bytes per edge of one launch unit of each tensor-track
    kind, from the staged per-unit figures: a non-final tensor product (or its
    adjoint) reads and writes one w x n FP32 feature row per edge (4 * 2 w n
    bytes; 4.6 KB for l_max 2, n 64); an environment scatter (or its adjoint)
    reads the (l_max + 1) n weights and the dim harmonics of each edge; the
    final layer's product reads one w x n row.  Per-centre rows (which stay
    in cache) are not counted."""
    n, D = mc.n_tensor, (mc.l_max + 1) ** 2
    w = D                                           # natural-parity features (two-layer models)
    tp = 4 * 2 * w * n
    env = 4 * ((mc.l_max + 1) * n + D)
    return {"env": env, "tp_mix": tp, "mix_adjoint": tp, "tp_env_adjoint": tp + env,
            "tp_env_adjoint_final": 4 * w * n + env}


def tensor_symbols(mc, bf3=True):
    """Kernel symbols (as rocprofv3 prints them) behind each timed tensor-track
    launch kind of one step: the layers' patterns TpPattern<l_max, input kind,
    output kind> (1 natural parity, 2 both parities, 0 the final scalar), the
    lane groups of the adjoint kernels (64 / n channels), for the first
    layer's adjoint the rank-1 form of its input, and for the tile kernels
    whether the mixing runs as BF16 x 3 (`bf3`, the BF16-mixed modes)."""
    nl, lm, G = mc.n_layers, mc.l_max, 64 // mc.n_tensor
    kin = [1 if (L == 0 or L == nl - 1) else 2 for L in range(nl)]
    kout = [0 if L == nl - 1 else (2 if nl >= 3 and L < nl - 2 else 1) for L in range(nl)]
    pat = lambda L: f"TpPattern<{lm}, {kin[L]}, {kout[L]}>"
    a0 = lambda L: "true" if L == 0 else "false"
    # the edge pass adds to dE/dY rows written before it: every layer but the
    # last (run first), and the last too when it is the rank-1 first layer
    keep = lambda L: "true" if (L < nl - 1 or L == 0) else "false"
    out = {"tp_env_adjoint_final": [f"k_tp_adjoint_gamma<{pat(nl - 1)}, {G}, {a0(nl - 1)}>",
                                    f"k_tp_adjoint_edges<{pat(nl - 1)}, {G}, {keep(nl - 1)}>"]}
    if nl > 1:
        b = "true" if bf3 else "false"
        out["tp_mix"] = [f"k_tp_mix<{pat(L)}, 16, {b}>" for L in range(nl - 1)]
        out["mix_adjoint"] = [f"k_mix_adjoint<{pat(L + 1)}, 16, {b}>" for L in range(nl - 1)]
        out["tp_env_adjoint"] = [s for L in range(nl - 1)
                                 for s in (f"k_tp_adjoint_gamma<{pat(L)}, {G}, {a0(L)}>",
                                           f"k_tp_adjoint_edges<{pat(L)}, {G}, {keep(L)}>")]
    return out


def run_gpu(mc, s, w, precision, steps, warmup, want_kernel_times, autotune=True):
    import torch
    import paper_2304_10061_amd as P
    import workloads as W
    dev = torch.device("cuda", 0)
    m = P.Model(P.config_from(mc, precision=precision), W.pack_weights(mc, w))
    pos = torch.as_tensor(s.pos, dtype=torch.float64, device=dev)
    sp = torch.as_tensor(s.species, dtype=torch.int32, device=dev)
    F = torch.empty((s.n_total, 3), dtype=torch.float64, device=dev)
    Ea = torch.empty(s.n_local, dtype=torch.float64, device=dev)
    vir = torch.empty(9, dtype=torch.float64, device=dev)
    E = torch.empty(1, dtype=torch.float64, device=dev)

    def step():
        m.neighbors(pos, sp, s.cell, s.pbc, s.n_local)
        m.energy_forces(pos, sp, F, atom_energy=Ea, virial=vir, energy=E)

    tiles = None
    if autotune:
        m.neighbors(pos, sp, s.cell, s.pbc, s.n_local)
        tiles = m.autotune(pos, sp)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # per-step events on the stream the library runs on (torch's current one)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record()
    for k in range(steps):
        step()
        evs[k + 1].record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    per_step = [evs[k].elapsed_time(evs[k + 1]) for k in range(steps)]
    # energy + forces alone on the same list (the list is rebuilt by every step above)
    ef = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    m.neighbors(pos, sp, s.cell, s.pbc, s.n_local)
    ef[0].record()
    for k in range(steps):
        m.energy_forces(pos, sp, F, atom_energy=Ea, virial=vir, energy=E)
        ef[k + 1].record()
    torch.cuda.synchronize()
    ef_ms = [ef[k].elapsed_time(ef[k + 1]) for k in range(steps)]
    res = {"ms_per_step": ms, "ms_per_step_median": float(np.median(per_step)),
           "ef_ms_median": float(np.median(ef_ms)), "edges": m.num_edges(), "energy": float(E.item()),
           "workspace_GB": m.workspace_bytes() / 1e9, "tiles": tiles}
    if want_kernel_times:
        m.set_timing(True)
        reps = 3
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        kt = m.kernel_times()
        m.set_timing(False)
        res["kernel_ms"] = {k: v[0] / reps for k, v in kt.items()}
        res["kernel_launches"] = {k: v[1] // reps for k, v in kt.items()}
        # the neighbour build alone (events on the same stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            m.neighbors(pos, sp, s.cell, s.pbc, s.n_local)
        ev[1].record()
        torch.cuda.synchronize()
        res["neighbors_ms"] = ev[0].elapsed_time(ev[1]) / reps
    m.close()
    return res


def cpu_baseline(mc, s, w, n_centres):
    import torch
    from oracle import model as OM
    from oracle.neighbors import neighbor_list
    cores = len(os.sched_getaffinity(0))
    torch.set_num_threads(cores)
    nbr = neighbor_list(s.pos, s.cell, s.pbc, mc.r_cut, method="kdtree")
    rng = np.random.default_rng(0)
    cents = np.sort(rng.choice(s.n_local, size=n_centres, replace=False))
    p = OM.Params(mc, w)
    # in pieces of 512 centres, so that host memory stays at a few GB
    t0 = time.perf_counter()
    for k in range(0, n_centres, 512):
        OM.evaluate_centres(mc, w, s, cents[k:k + 512], nbr, params=p)
    t = time.perf_counter() - t0
    return {"value": n_centres / t, "unit": "atom-steps/s", "cores": int(torch.get_num_threads()),
            "kind": "oracle",
            "sample": f"{n_centres} random centres of the same box (their {int(np.sum(np.isin(nbr[0], cents)))} "
                      f"edges, energy + edge gradients in FP64), {t:.1f} s"}


def deep_workload_line(steps, warmup, cpu_sample, no_cpu):
    """The deeper tensor track (three layers, l_max 3: unnatural-parity
    irreps and l = 3 harmonics) on the 3,000-atom water box."""
    import paper_2304_10061_amd as P
    import workloads as W
    mc, s, w = W.deep_workload()
    info = P.describe(P.config_from(mc))
    bf = run_gpu(mc, s, w, HEADLINE_PREC, steps, warmup, want_kernel_times=True)
    fp = run_gpu(mc, s, w, 0, max(3, steps // 2), min(2, warmup), want_kernel_times=True)
    kms = bf["kernel_ms"]
    macs = mlp_macs_per_edge(mc)
    tfl = tensor_flops_per_edge(mc, info)
    dom = max(kms, key=kms.get)
    E = bf["edges"]
    if dom in macs:
        flops = 2.0 * macs[dom] * E * bf["kernel_launches"].get(dom, 1)
        roof = {"kernel": dom, "bound": "mfma", "peak": BF16_PEAK_TFLOPS}
    else:
        flops = float(tfl.get(dom, 0)) * E
        roof = {"kernel": dom, "bound": "alu", "peak": FP32_PEAK_TFLOPS}
    achieved = flops / (kms[dom] * 1e-3) / 1e12
    launches = max(1, bf["kernel_launches"].get(dom, 1))
    syms = tensor_symbols(mc).get(dom)
    traffic = None
    if syms:
        per = [traffic_per_launch(sym, TRAFFIC_SUMMARY_DEEP) for sym in syms]
        traffic = sum(per) / launches if all(v is not None for v in per) else None
    roof.update({"achieved": achieved, "unit": "TFLOP/s", "frac": achieved / roof["peak"], "traffic": traffic,
                 "symbols": syms, "flops_per_launch": flops / launches, "avg_launch_ms": kms[dom] / launches})
    if traffic is not None:
        # the same launch against the HBM roof on its measured traffic
        roof["hbm_frac_traffic"] = traffic / (kms[dom] / launches * 1e-3) / (HBM_PEAK_GBS * 1e9)
    tensor = {k: {"ms": round(kms[k], 4), "tflops": float(tfl[k]) * E / (kms[k] * 1e-3) / 1e12}
              for k in tfl if k in kms}
    out = {
        "metric": "atom-steps/s (E+forces), 3,000-atom water box, three-layer l_max 3 model",
        "value": s.n_local / (bf["ms_per_step"] * 1e-3), "unit": "atom-steps/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": bf["ms_per_step"],
        "ms_per_step_median": bf["ms_per_step_median"],
        "energy_forces_only": {"ms_median": bf["ef_ms_median"], "value": s.n_local / (bf["ef_ms_median"] * 1e-3)},
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "water-like periodic box: 3000 atoms, 31.1 A cube, H:O 2:1, jittered lattice "
                               "+-0.4 A, r_c 4 A; Allegro l_max 3, 3 layers (unnatural-parity irreps in the "
                               "middle layer), 32 tensor channels, latent MLP [128,128], edge MLP [128]; "
                               "random weights",
                   "atoms": int(s.n_local), "edges": int(E),
                   "paths_per_layer": [int(info.n_paths[k]) for k in range(mc.n_layers)],
                   "nonzeros_per_layer": [int(info.n_nonzero[k]) for k in range(mc.n_layers)],
                   "parallelism": "single GPU"},
        "roofline": roof,
        "tensor_track": tensor,
        "fp32": {"value": s.n_local / (fp["ms_per_step"] * 1e-3), "ms_per_step": fp["ms_per_step"],
                 "energy_bf16_minus_fp32_per_atom": (bf["energy"] - fp["energy"]) / s.n_local},
        "kernel_ms": {k: round(v, 4) for k, v in sorted(kms.items(), key=lambda kv: -kv[1])},
        "neighbors_ms": bf["neighbors_ms"], "workspace_GB": bf["workspace_GB"], "tiles": bf["tiles"],
        "source_hash": kernel_source_hash(),
    }
    if not no_cpu:
        out["cpu_baseline"] = cpu_baseline(mc, s, w, min(cpu_sample, s.n_local))
    return out


MD_SIGMA = 0.02
MD_CLUSTER_SKIN = 0.5   # lists of up to one evaluation chunk are rebuilt inside the step graph
HEADLINE_PREC = 3   # ALLEGRO_PREC_BF16_MIXED


def md_workload(kind, steps, warmup, dt_fs, precision=HEADLINE_PREC):
    """One GPU's MD share: the 1M-atom subdomain with its ghost shell (a list
    of several evaluation chunks, rebuilt by the host when an atom has moved
    half the skin), or 512 uneven clusters in one batched evaluation (every
    step, neighbour rebuild included, a replay of one captured hipGraph)."""
    import torch
    import paper_2304_10061_amd as P
    import workloads as W
    dev = torch.device("cuda", 0)
    cfg = 4 if kind == "subdomain" else 5
    mc = W.model_config(cfg)
    w = W.make_weights(mc, W.seeds(cfg)[3])
    t_gen = time.perf_counter()
    if kind == "subdomain":
        base = W.jittered_lattice_box(1_000_000, 215.0, 0.5, W.PROTEIN_MIX, 4, sites_per_side=100)
        sysm = W.ghost_shell(base, 6.0)
        skin = 0.3
        chunk = 8_000_000
        masses = base.masses
    else:
        sysm = W.clusters(512, 5)
        skin = MD_CLUSTER_SKIN
        chunk = 0
        masses = sysm.masses
    t_gen = time.perf_counter() - t_gen
    nl = sysm.n_local
    free0, total = torch.cuda.mem_get_info()
    # The random-weight model is far from equilibrium on these structures
    # (forces of order 0.5 eV/A at sigma = 1); per-species energy scales of
    # MD_SIGMA keep forces near thermal magnitude so that the neighbour skin
    # stays valid over the run.  The cost of a step does not depend on sigma.
    sig = np.full(mc.n_species, MD_SIGMA)
    m = P.Model(P.config_from(mc, precision=precision, edge_chunk=chunk, neighbor_skin=skin), W.pack_weights(mc, w),
                sig, np.zeros(mc.n_species))
    pos = torch.as_tensor(sysm.pos, dtype=torch.float64, device=dev)
    sp = torch.as_tensor(sysm.species, dtype=torch.int32, device=dev)
    vel = torch.as_tensor(W.maxwell_boltzmann(masses, 300.0, W.seeds(cfg)[4]), dtype=torch.float64, device=dev)
    mass = torch.as_tensor(masses, dtype=torch.float64, device=dev)
    F = torch.zeros((sysm.n_total, 3), dtype=torch.float64, device=dev)
    n_total_steps = warmup + steps
    thermo = torch.zeros((n_total_steps, 2), dtype=torch.float64, device=dev)

    def build():
        if kind == "subdomain":
            return m.neighbors(pos, sp, sysm.cell, sysm.pbc, nl)
        return m.neighbors_batched(sysm.atom_offsets, pos, sp)

    if kind == "subdomain":
        own = sysm.ghost_owner
        m.set_ghosts(nl, own, sysm.pos[nl:] - base.pos[own])
    e_first = build()
    tiles = m.autotune(pos, sp)   # edge-tile shapes for this system (a few evaluations)
    # warm-up steps (the first call captures the step graph), then the timed
    # steps in one call: the list is rebuilt inside the steps whenever an
    # atom has moved half the skin since the last build
    use_graph = kind == "clusters"
    vir = torch.zeros((n_total_steps, 9), dtype=torch.float64, device=dev)
    _, over_warm = m.md_run_all(warmup, dt_fs, mass, pos, vel, F, sp, thermo=thermo[:warmup], init_forces=True,
                                use_graph=use_graph, virial=vir[:warmup])
    captures_warm = m.md_stats()[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    disp, over_timed = m.md_run_all(steps, dt_fs, mass, pos, vel, F, sp, thermo=thermo[warmup:], use_graph=use_graph,
                                    virial=vir[warmup:])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    captures, capacity, dev_rebuild, rebuilds = m.md_stats()
    free1, _ = torch.cuda.mem_get_info()
    th = thermo.cpu().numpy()
    etot = th[:, 0] + th[:, 1]
    ms = elapsed * 1e3 / steps
    out = {
        "metric": "atom-steps/s (E+forces+FP64 velocity Verlet)",
        "value": nl / (ms * 1e-3), "unit": "atom-steps/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": ("1,000,000-atom protein-like subdomain (215 A) + 6 A periodic-image ghost shell, "
                                "model r_c 4 A, n 32, latent [128,128], list in 8M-edge chunks rebuilt by the host "
                                "when an atom has moved half the skin"
                                if kind == "subdomain" else
                                "512 non-periodic clusters (20-2000 atoms, log-uniform), batched; each step, neighbour "
                                "rebuild on the device included, is a replay of one captured hipGraph"),
                   "atoms": int(nl), "ghosts": int(sysm.n_total - nl), "dt_fs": dt_fs,
                   "neighbor_skin": skin, "edges_first_build": int(e_first), "edges_last_build": int(m.num_edges())},
        "peak_hbm_GB": (free0 - free1) / 1e9,
        "library_workspace_GB": m.workspace_bytes() / 1e9,
        "energy_drift_per_atom": float((etot[-1] - etot[0]) / nl),
        # per-step FP64 virial (eV): its trace at the last step and the mean over the timed steps
        "virial_trace_last_step": float(np.trace(vir[-1].cpu().numpy().reshape(3, 3))),
        "virial_trace_mean_timed": float(np.mean([np.trace(r.reshape(3, 3)) for r in vir[warmup:].cpu().numpy()])),
        "energy_fluct_per_atom": float(np.std(etot) / nl),
        "species_energy_scale": MD_SIGMA,
        "neighbor_rebuilds_timed_last_call": int(rebuilds), "rebuilds_on_device": bool(dev_rebuild),
        "edge_capacity": int(capacity), "graph_captures": int(captures),
        "capacity_overflows": {"warmup": over_warm, "timed": over_timed},
        "graph_captures_during_timed_steps": int(captures - captures_warm),
        "max_displacement_since_last_rebuild": disp,
        "tiles": tiles, "setup_s": t_gen, "source_hash": kernel_source_hash(),
    }
    m.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=4096,
                    help="centres of the box in the oracle timing sample (about 10 s on 16 cores)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 and single-rounded BF16 comparisons")
    ap.add_argument("--workload", default="protein-box", choices=["protein-box", "subdomain", "clusters", "deep"],
                    help="protein-box (default, the headline); subdomain / clusters run MD; deep = three-layer "
                         "l_max 3 model on the 3,000-atom water box")
    ap.add_argument("--dt", type=float, default=1.0, help="MD time step (fs) for the MD workloads")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="run a plain copy of this many MiB first (counter calibration under rocprofv3 --pmc)")
    ap.add_argument("--summarize", nargs=4, metavar=("STATS_DIR", "FETCH_DIR", "WRITE_DIR", "BENCH_LOG"),
                    help="print the markdown summary of rocprofv3 outputs (and the profiled run's output) and exit")
    ap.add_argument("--command", action="append", default=[], help="profiling command (for --summarize)")
    ap.add_argument("--summarize-mfma", default=None, metavar="MFMA_DIR",
                    help="--pmc run of SQ_VALU_MFMA_BUSY_CYCLES and SQ_INSTS_VALU_MFMA_MOPS_BF16 (for --summarize)")
    args = ap.parse_args()
    if args.summarize:
        print(summarize_profiles(*args.summarize, args.calibration_copy_mib, args.command, args.summarize_mfma))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the energy/force path runs on a single MI355X "
              "(spatial decomposition across GPUs is not implemented here)", file=sys.stderr)
        sys.exit(2)

    if args.calibration_copy_mib:
        calibration_copy(args.calibration_copy_mib)
    if args.workload == "deep":
        print(json.dumps(deep_workload_line(args.steps, args.warmup, min(args.cpu_sample, 512),
                                            args.no_cpu_baseline)), flush=True)
        return
    if args.workload != "protein-box":
        print(json.dumps(md_workload(args.workload, args.steps, args.warmup, args.dt)), flush=True)
        return

    import workloads as W
    mc, s, w = W.workload(3)
    bf = run_gpu(mc, s, w, HEADLINE_PREC, args.steps, args.warmup, want_kernel_times=True)
    fp = None if args.no_fp32 else run_gpu(mc, s, w, 0, max(3, args.steps // 4), min(2, args.warmup), True)
    bs = None if args.no_fp32 else run_gpu(mc, s, w, 2, max(3, args.steps // 2), min(2, args.warmup), True)
    bp = None if args.no_fp32 else run_gpu(mc, s, w, 1, max(3, args.steps // 2), min(2, args.warmup), True)
    # the same box with the paper's per-ordered-species-pair cutoffs (BF16_MIXED)
    mcp = copy.copy(mc)
    mcp.pair_cutoffs = W.paper_pair_cutoffs(mc.n_species, mc.r_cut)
    pc = None if args.no_fp32 else run_gpu(mcp, s, w, HEADLINE_PREC, max(3, args.steps // 2), min(2, args.warmup),
                                           False)
    # the same box with the ZBL pair term (atomic numbers H 1, C 6, N 7, O 8)
    mcz = copy.copy(mc)
    mcz.atomic_numbers = W.atomic_numbers(mc.n_species)
    zb = None if args.no_fp32 else run_gpu(mcz, s, w, HEADLINE_PREC, max(3, args.steps // 2), min(2, args.warmup),
                                           False)

    value = s.n_local / (bf["ms_per_step"] * 1e-3)
    macs = mlp_macs_per_edge(mc)
    kms = bf["kernel_ms"]
    dom = max(kms, key=kms.get)
    roof = None
    if dom in macs:
        flops = 2.0 * macs[dom] * bf["edges"] * bf["kernel_launches"].get(dom, 1)
        achieved = flops / (kms[dom] * 1e-3) / 1e12
        sym = mlp_symbol(dom, 1, (bf["tiles"] or {}).get(dom, 0), mc.latent)
        launches = max(1, bf["kernel_launches"].get(dom, 1))
        avg_ms = kms[dom] / launches
        io_bytes = mlp_bytes_per_edge(mc)[dom] * bf["edges"]   # per launch (one launch per chunk)
        roof = {"kernel": dom, "symbol": sym, "bound": "mfma", "achieved": achieved, "peak": BF16_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / BF16_PEAK_TFLOPS, "traffic": traffic_per_launch(sym),
                "flops_per_launch": flops / launches, "avg_launch_ms": avg_ms,
                # the same launch against the HBM roof, on the bytes this
                # kernel design itself stages (its input and output rows)
                "staged_io_bytes_per_launch": io_bytes / launches,
                "hbm_frac_staged_io": io_bytes / launches / (avg_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
                "mfma_counters": mfma_busy_counters([sym])}
    elif dom in tensor_bytes_per_unit(mc) and mc.n_layers == 2:
        # a staged tensor-track unit: HBM-bound (its FP32 arithmetic is ~25 flop per
        # byte moved, near the FP32 ridge), measured against 8 TB/s on the
        # algorithmic bytes of one launch unit
        launches = max(1, bf["kernel_launches"].get(dom, 1))
        avg_ms = kms[dom] / launches
        unit_bytes = tensor_bytes_per_unit(mc)[dom] * bf["edges"]
        achieved = unit_bytes / (avg_ms * 1e-3) / 1e9
        syms = tensor_symbols(mc).get(dom, [])
        per = [traffic_per_launch(sym) for sym in syms]
        traffic = sum(per) / launches if syms and all(v is not None for v in per) else None
        roof = {"kernel": dom, "symbols": syms, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "bytes_per_launch": unit_bytes, "avg_launch_ms": avg_ms}
        if traffic is not None:
            roof["hbm_frac_traffic"] = traffic / (avg_ms * 1e-3) / (HBM_PEAK_GBS * 1e9)
        info = P_describe(mc)
        if info is not None:
            tfl = tensor_flops_per_edge(mc, info).get(dom)
            if tfl:
                # the same unit against the FP32 vector roof
                roof["alu_frac"] = tfl * bf["edges"] / (avg_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": 8000.0, "unit": "GB/s",
                "frac": None, "traffic": None}
    # whole-step MLP-GEMM MFMA utilisation
    mlp_ms = sum(v for k, v in kms.items() if k in macs)
    mlp_flops = 2.0 * sum(macs.values()) * bf["edges"]
    out = {
        "metric": "atom-steps/s (E+forces), 23.5k-atom protein-like box, FP32 vs BF16-MFMA",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": bf["ms_per_step"],
        "ms_per_step_median": bf["ms_per_step_median"],
        "energy_forces_only": {"ms_median": bf["ef_ms_median"],
                               "value": s.n_local / (bf["ef_ms_median"] * 1e-3)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "protein-like periodic box: 23558 atoms, 61.76 A cube, H:C:N:O 50:30:8:12, "
                               "jittered lattice +-0.5 A, r_c 6 A; Allegro l_max 2, 2 layers, 64 tensor "
                               "channels, latent MLP [256,256,256], edge MLP [128]; random weights",
                   "atoms": int(s.n_local), "edges": int(bf["edges"]), "global_batch": int(s.n_local),
                   "parallelism": "single GPU"},
        "roofline": roof,
        "mlp_gemm": {"tflops": mlp_flops / (mlp_ms * 1e-3) / 1e12 if mlp_ms else None,
                     "mfma_frac": (mlp_flops / (mlp_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS) if mlp_ms else None,
                     "ms": mlp_ms,
                     # matrix-core busy fraction and executed rate from the
                     # committed counter summary (weight pairs and the
                     # backward's recomputation included)
                     "mfma_counters": mfma_busy_counters(
                         [mlp_symbol(k, 1, (bf["tiles"] or {}).get(k, 0), mc.latent) for k in macs])},
        "kernel_ms": {k: round(v, 4) for k, v in sorted(kms.items(), key=lambda kv: -kv[1])},
        "neighbors_ms": bf["neighbors_ms"],
        "workspace_GB": bf["workspace_GB"],
        "source_hash": kernel_source_hash(),
    }
    out["precision_mode"] = ("BF16 MFMA, FP32 accumulation; BF16 weight pairs (hi + lo) in the two-body MLP "
                             "and the first layer of each later MLP, single-rounded elsewhere")
    if fp is not None:
        out["fp32"] = {"value": s.n_local / (fp["ms_per_step"] * 1e-3), "ms_per_step": fp["ms_per_step"],
                       "mlp_gemm_ms": sum(v for k, v in fp["kernel_ms"].items() if k in macs),
                       "energy_bf16_minus_fp32_per_atom": (bf["energy"] - fp["energy"]) / s.n_local}
        out["bf16_speedup_vs_fp32"] = fp["ms_per_step"] / bf["ms_per_step"]
        out["energy_minus_fp32_per_atom"] = (bf["energy"] - fp["energy"]) / s.n_local
    if bs is not None:
        out["bf16_single_rounded_weights"] = {
            "value": s.n_local / (bs["ms_per_step"] * 1e-3), "ms_per_step": bs["ms_per_step"],
            "mlp_gemm_ms": sum(v for k, v in bs["kernel_ms"].items() if k in macs),
            "energy_minus_fp32_per_atom": (bs["energy"] - fp["energy"]) / s.n_local}
    if bp is not None:
        out["bf16_all_weight_pairs"] = {
            "value": s.n_local / (bp["ms_per_step"] * 1e-3), "ms_per_step": bp["ms_per_step"],
            "mlp_gemm_ms": sum(v for k, v in bp["kernel_ms"].items() if k in macs),
            "energy_minus_fp32_per_atom": (bp["energy"] - fp["energy"]) / s.n_local, "tiles": bp["tiles"]}
    if pc is not None:
        out["pair_cutoffs"] = {
            "cutoffs": "H-H 3.0, H-C 1.25, H-O 1.25, O-H 3.0 A (ordered: centre-neighbour); others %.1f A" % mc.r_cut,
            "value": s.n_local / (pc["ms_per_step"] * 1e-3), "ms_per_step": pc["ms_per_step"],
            "edges": pc["edges"], "edges_single_cutoff": bf["edges"],
            "speedup_vs_single_cutoff": bf["ms_per_step"] / pc["ms_per_step"], "tiles": pc["tiles"]}
    if zb is not None:
        out["zbl"] = {"value": s.n_local / (zb["ms_per_step"] * 1e-3), "ms_per_step": zb["ms_per_step"],
                      "overhead_vs_plain": zb["ms_per_step"] / bf["ms_per_step"] - 1.0}
    out["tiles"] = bf["tiles"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mc, s, w, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
