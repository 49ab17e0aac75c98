"""Builds libhcao.so (the gfx950 HIP kernels and the host runtime) in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libhcao.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("HCAO_ARCH", "gfx950")
# IEEE fp64 without contraction (the oracle parity contract), no packed fp32
COMMON = ["-O3", "-fPIC", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-Wall",
          "-I", INCLUDE, "-I", CSRC]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    k_obj = os.path.join(BUILD, "hcao_kernels.o")
    r_obj = os.path.join(BUILD, "hcao_runtime.o")
    _run([HIPCC, "-x", "hip", *DEVICE, *COMMON, "-c", os.path.join(CSRC, "hcao_kernels.hip"), "-o", k_obj])
    _run([HIPCC, *COMMON, "-c", os.path.join(CSRC, "hcao_runtime.cpp"), "-o", r_obj])
    tmp = LIB + ".tmp"
    _run([HIPCC, *DEVICE, "-shared", "-fPIC", "-o", tmp, k_obj, r_obj])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
