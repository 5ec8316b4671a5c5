"""Build libcsc.so for gfx950 with hipcc (in-tree, no JIT cache).

    python -m paper_1602_02018_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "libcsc.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CSC_CXX", "/opt/rocm/llvm/bin/clang++")
ARCH = "gfx950"

SOURCES = {
    "kernels.hip": [],
    "api.hip": [],
    "batched.hip": [],
    "api_batched.hip": [],
    "mlp.hip": [],
    "order.hip": [],
    "block.hip": [],
    "kmeans.hip": ["-ffp-contract=off"],
    "kmeans_gpu.hip": ["-ffp-contract=off"],
}

# host-only C++ (no device code), compiled by the host compiler
HOST_SOURCES = {
    "dense.cpp": ["-ffp-contract=off"],
}
HOST_COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall"]

COMMON = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions are disabled for every HIP translation unit
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall",
    "-Wno-unused-result",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}")
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    jobs = []
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES) + len(HOST_SOURCES)) as ex:
        for src, extra in SOURCES.items():
            obj = os.path.join(BUILD, src.replace(".hip", ".o"))
            objs.append(obj)
            cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(HERE, "csrc", src), "-o", obj]
            jobs.append(ex.submit(_run, cmd, verbose))
        for src, extra in HOST_SOURCES.items():
            obj = os.path.join(BUILD, src.replace(".cpp", ".o"))
            objs.append(obj)
            cmd = [CXX, *HOST_COMMON, *extra, "-c", os.path.join(HERE, "csrc", src), "-o", obj]
            jobs.append(ex.submit(_run, cmd, verbose))
        for j in jobs:
            j.result()
    tmp = OUT + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
