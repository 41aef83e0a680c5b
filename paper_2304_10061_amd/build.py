"""Build liballegro_mi355x.so (gfx950) in-tree with hipcc.

Every source under csrc/ is compiled to an object in _build/ (in parallel) and
linked into paper_2304_10061_amd/liballegro_mi355x.so.  Run as
`python -m paper_2304_10061_amd.build` or call `build()`.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liballegro_mi355x.so")
ARCH = "gfx950"

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # MFMA accumulators in ordinary VGPRs: avoids AGPR<->VGPR copies of
         # the accumulators around the GEMM loops
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         # the coupling tables of the larger patterns are evaluated at compile time
         "-fconstexpr-steps=200000000",
         "-Wno-unused-result"]

SOURCES = ["abi.cpp", "neighbors.hip", "edge.hip", "mlp.hip", "mlp_fp32.hip", "mlp_bf16.hip", "mlp_bf16s.hip",
           "mlp_rr1f.hip", "mlp_rr1b.hip", "mlp_rr2f.hip", "mlp_rr2b.hip", "tensor.hip", "md.hip"]


def _hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found")
    return path


def _compile(src: str) -> str:
    obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
