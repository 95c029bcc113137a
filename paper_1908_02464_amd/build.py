"""Build the gfx950 shared library libweno_l2is.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libweno_l2is.so")
# (source, FMA contraction).  The sweep kernels, shared by the single-grid
# 1D/2D path and the batched form, contract only inside one expression, so
# their arithmetic follows the source and does not depend on the kernel they
# are inlined into: a grid gives the same bits on both paths.  The fused 3D
# kernels also contract across statements (fewer FP64 instructions).
SOURCES = [("wl2_capi.hip", "on"), ("wl2_batch.hip", "on"), ("wl2_fused3d.hip", "fast")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def compile_flags(src: str) -> list:
    """The hipcc flags one source is compiled with."""
    return HIPCC_FLAGS + [f"-ffp-contract={dict(SOURCES)[src]}"]


def build(verbose: bool = True) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs, procs = [], []
    for src, contract in SOURCES:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = ([hipcc] + HIPCC_FLAGS + [f"-ffp-contract={contract}", "-I", os.path.join(ROOT, "include"),
               "-c", "-o", obj, os.path.join(PKG, "csrc", src)])
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [src for src, pr in procs if pr.wait() != 0]
    if failed:
        raise RuntimeError("hipcc failed on " + ", ".join(failed))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
