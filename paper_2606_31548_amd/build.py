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


# instrumented build: per-phase clock sums of the step kernel (hcao_phase_clocks)
LIB_CLOCKS = os.path.join(HERE, "libhcao_clocks.so")


def build(verbose: bool = True, phase_clocks: bool = False) -> str:
    """Compiles the library in-tree. phase_clocks: the instrumented variant
    libhcao_clocks.so (load it with HCAO_LIBRARY=<path>)."""
    os.makedirs(BUILD, exist_ok=True)
    tag = "_clocks" if phase_clocks else ""
    defs = ["-DHCAO_PHASE_CLOCKS"] if phase_clocks else []
    lib = LIB_CLOCKS if phase_clocks else LIB
    k_obj = os.path.join(BUILD, f"hcao_kernels{tag}.o")
    r_obj = os.path.join(BUILD, f"hcao_runtime{tag}.o")
    t_obj = os.path.join(BUILD, f"hcao_host_tables{tag}.o")
    _run([HIPCC, "-x", "hip", *DEVICE, *COMMON, *defs, "-c", os.path.join(CSRC, "hcao_kernels.hip"), "-o", k_obj])
    _run([HIPCC, *DEVICE, *COMMON, *defs, "-c", os.path.join(CSRC, "hcao_runtime.cpp"), "-o", r_obj])
    _run([HIPCC, *DEVICE, *COMMON, "-c", os.path.join(CSRC, "hcao_host_tables.cpp"), "-o", t_obj])
    tmp = lib + ".tmp"
    _run([HIPCC, *DEVICE, "-shared", "-fPIC", "-o", tmp, k_obj, r_obj, t_obj])
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(phase_clocks="--phase-clocks" in sys.argv[1:])
    sys.exit(0)
