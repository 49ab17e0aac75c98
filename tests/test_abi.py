"""The C ABI library loads on a CPU-only host and exports every function that
include/hcao.h declares (no compute calls: those need the GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hcao.h")
LIB = os.path.join(ROOT, "paper_2606_31548_amd", "libhcao.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hcao_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("hcao_create", "hcao_add_species", "hcao_add_reaction", "hcao_finalize", "hcao_load_particles",
                 "hcao_init_thermal", "hcao_step", "hcao_read_moments", "hcao_read_reaction_counts",
                 "hcao_destroy"):
        assert want in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhcao.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhcao.so not built")
def test_status_strings_without_device():
    lib = ctypes.CDLL(LIB)
    lib.hcao_status_string.restype = ctypes.c_char_p
    lib.hcao_status_string.argtypes = [ctypes.c_int]
    assert lib.hcao_status_string(0) == b"ok"
    assert lib.hcao_status_string(-5) == b"cell capacity exceeded"


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    from paper_2606_31548_amd import hcao
    monkeypatch.setattr(hcao, "_lib", None)
    monkeypatch.setattr(hcao, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        hcao.load_library()
