"""Build ``libgi.so`` (the gfx950 HIP kernels and the C ABI of include/gi.h) in place.

hipcc cross-compiles for gfx950 without a GPU.  Packed FP32 instructions are disabled on
purpose (``-packed-fp32-ops``): the kernels are written for one FP32 lane per value.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libgi.so")
SOURCES = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
# the roofline microbenchmarks: a library of their own, loaded only by the benchmark
PEAKS_LIB = os.path.join(HERE, "libgi_peaks.so")
PEAKS_SOURCES = [os.path.join(HERE, "peaks", "k_peaks.hip")]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    _build_one(SOURCES, LIB, verbose)
    _build_one(PEAKS_SOURCES, PEAKS_LIB, verbose)
    return LIB


def _build_one(sources, lib, verbose):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = lib + f".tmp{os.getpid()}"
    cmd = [hipcc, *FLAGS, *sources, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    errs = [ln for ln in res.stderr.splitlines()
            if "packed-fp32-ops' is not a recognized feature" not in ln]
    if res.returncode != 0:
        sys.stderr.write("\n".join(errs) + "\n")
        raise RuntimeError(f"hipcc failed building {os.path.basename(lib)}")
    if verbose and errs:
        sys.stderr.write("\n".join(errs) + "\n")
    os.replace(tmp, lib)


if __name__ == "__main__":
    print(build(verbose=True))
