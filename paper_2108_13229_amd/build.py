"""Build the HIP library libsd.so for gfx950 in-tree.

Usage: python -m paper_2108_13229_amd.build   (or import and call build()).
Host code is compiled without floating-point contraction so that the
assembled matrix and the AMG hierarchy are reproducible bit-for-bit.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libsd.so")
BUILD = os.path.join(HERE, "_build")

HIP_SOURCES = ["kernels.hip"]
CPP_SOURCES = ["assemble.cpp", "assemble3d.cpp", "amg_setup.cpp", "ilu.cpp", "solver.cpp", "api.cpp", "dn.cpp", "server.cpp"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-I" + INCLUDE, "-I" + CSRC, "-Wall",
          "-Wno-unused-function"]
# Packed FP32 arithmetic is disabled for device code.
GPU = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
       "-munsafe-fp-atomics"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("compile failed: " + cmd[-1])
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run(["hipcc", "-c", *COMMON, *GPU, "-x", "hip", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in CPP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run(["hipcc", "-c", *COMMON, "-ffp-contract=off", "-x", "c++",
              "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run(["hipcc", "-shared", "--offload-arch=gfx950", *objs, "-o", tmp, "-lpthread",
          "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
