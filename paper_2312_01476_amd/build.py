"""Build the gfx950 HIP library ``libejoin.so`` in-tree.

Every source under ``csrc/`` is compiled by hipcc for gfx950 and linked into
one shared library next to this file.  The FP64 rescore source is compiled
without floating-point contraction so that its arithmetic is exactly the
canonical sequential rule.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libejoin.so")
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
          "-I", os.path.join(ROOT, "include"), "-Wall",
          # packed FP32 instructions are kept out of every kernel
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
PER_FILE = {
    "rescore.hip": ["-ffp-contract=off"],
    "topk.hip": ["-ffp-contract=off"],
    # accumulators of the panel kernel are always finite: IEEE mode off lets
    # min/max skip NaN canonicalisation in the threshold screening
    "panel.hip": ["-mno-amdgpu-ieee", "-fno-honor-nans"],
}
SOURCES = ["prep.hip", "gemm_threshold.hip", "panel.hip", "rescore.hip", "topk.hip", "batch.hip",
           "select.hip", "nlj.hip", "prune.hip",
           "mlp.hip", "prefilter.hip", "api.cpp", "api_batch.cpp", "api_mlp.cpp", "tune.cpp"]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *COMMON, *PER_FILE.get(src, []), "-x", "hip", "-c",
           os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
