"""Build of the gfx950 shared library libtvs.so (hipcc, in-tree).

Every HIP source is compiled for gfx950 only, with packed-FP32 instructions
disabled; the kernels are compiled without multiply-add contraction so
their float64 arithmetic (voxel decisions in particular) follows the written
order of operations.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libtvs.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = {
    "rows.hip": ["-ffp-contract=off"],
    "drop.hip": ["-ffp-contract=off"],
    "tv.hip": ["-ffp-contract=off"],
    "batch.hip": ["-ffp-contract=off"],
    "fbp.hip": ["-ffp-contract=off"],
    "serve.cpp": ["-x", "hip"],
    "tvs_api.cpp": ["-x", "hip"],
}
COMMON = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", INCLUDE, "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    """Compile every source and link libtvs.so; returns its path."""
    os.makedirs(LIBDIR, exist_ok=True)
    objs = []
    for src, extra in SOURCES.items():
        obj = os.path.join(LIBDIR, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
