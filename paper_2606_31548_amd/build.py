"""Builds libhcao.so (the gfx950 HIP kernels and the host runtime) in-tree,
and beside it two debugging forms of the same sources: libhcao_clocks.so
(per-phase clock sums of the step kernel, hcao_phase_clocks) and
libhcao_checked.so (every particle-slot and per-pair record index the
kernels form is checked against its array; a failure is reported as
HCAO_EBOUNDS). Load a debugging form with HCAO_LIBRARY=<path>."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

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
# roctx ranges around the runtime's host-side phases (rocprofv3 --marker-trace shows them)
LINK = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]

# the library forms: file name, preprocessor definitions
FORMS = {
    "product": ("libhcao.so", []),
    "clocks": ("libhcao_clocks.so", ["-DHCAO_PHASE_CLOCKS"]),
    "checked": ("libhcao_checked.so", ["-DHCAO_CHECKED"]),
}
LIB_CLOCKS = os.path.join(HERE, FORMS["clocks"][0])
LIB_CHECKED = os.path.join(HERE, FORMS["checked"][0])


def _run(cmd, verbose=True):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build_form(form: str = "product", verbose: bool = True) -> str:
    """Compiles one form of the library (see FORMS) in-tree; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    name, defs = FORMS[form]
    lib = os.path.join(HERE, name)
    tag = "" if form == "product" else "_" + form
    k_obj = os.path.join(BUILD, f"hcao_kernels{tag}.o")
    r_obj = os.path.join(BUILD, f"hcao_runtime{tag}.o")
    t_obj = os.path.join(BUILD, f"hcao_host_tables{tag}.o")
    _run([HIPCC, "-x", "hip", *DEVICE, *COMMON, *defs, "-c", os.path.join(CSRC, "hcao_kernels.hip"), "-o", k_obj],
         verbose)
    _run([HIPCC, *DEVICE, *COMMON, *defs, "-c", os.path.join(CSRC, "hcao_runtime.cpp"), "-o", r_obj], verbose)
    _run([HIPCC, *DEVICE, *COMMON, "-c", os.path.join(CSRC, "hcao_host_tables.cpp"), "-o", t_obj], verbose)
    tmp = lib + ".tmp"
    _run([HIPCC, *DEVICE, "-shared", "-fPIC", "-o", tmp, k_obj, r_obj, t_obj, *LINK], verbose)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = True, phase_clocks: bool = False, forms=None) -> str:
    """Compiles the library in-tree: by default every form at once (product,
    clocks, checked, each in compiler processes of its own); phase_clocks=True
    builds only the instrumented form. Returns the product library's path
    (the instrumented one's with phase_clocks=True)."""
    if phase_clocks:
        return build_form("clocks", verbose)
    forms = list(forms or FORMS)
    with ThreadPoolExecutor(max_workers=len(forms)) as ex:
        paths = dict(zip(forms, ex.map(lambda f: build_form(f, verbose), forms)))
    return paths.get("product", next(iter(paths.values())))


if __name__ == "__main__":
    build(phase_clocks="--phase-clocks" in sys.argv[1:])
    sys.exit(0)
