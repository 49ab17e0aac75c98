"""The bounds-checked form of the library (libhcao_checked.so): the same
kernels with every particle-slot and per-pair record index checked against
its array. It runs the parity cases of tests/checked_parity.py in a process
of its own (a process loads one form of the library) and must report no
index outside its array and stay bitwise equal to the oracle."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(ROOT, "paper_2606_31548_amd", "libhcao_checked.so")


def test_checked_build_runs_clean_and_bitwise():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} is missing: build it with __graft_entry__.build()")
    env = dict(os.environ, HCAO_LIBRARY=LIB)
    r = subprocess.run([sys.executable, "-u", os.path.join(HERE, "checked_parity.py")], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "checked ok" in r.stdout, out[-4000:]
