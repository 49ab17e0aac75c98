"""Host logic of bench.py (no GPU): the algorithmic-bytes count the roofline
rests on, the refusal of more than one GPU, the gate that ties measured
traffic to the kernel sources it was measured on, the workloads it names
and the oracle baseline's report."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2606_31548_amd import workloads as W  # noqa: E402


def test_algorithmic_bytes_counts_each_particles_state_once():
    """Per particle: velocity (3 b_v), species byte, 2 bytes per mode, 8 for
    a rotor, read and written; 64 B per cell. The spatial mode adds the
    24-byte position and moves the whole state a second time."""
    sp = [W.Species("atom", 1 * W.AMU), W.Species("tri", 30 * W.AMU, bend_theta_K=[900.0],
                                                  omega_e_per_m=[2e5, 2e5], chi_e=[0.01, 0.01], De_J=[8e-19] * 2)]
    counts = np.array([10.0, 5.0])
    assert bench.algorithmic_bytes(sp, counts, 3, b_v=8) == 10 * 2 * 25 + 5 * 2 * 31 + 64 * 3
    assert bench.algorithmic_bytes(sp, counts, 3, b_v=4) == 10 * 2 * 13 + 5 * 2 * 19 + 64 * 3
    sp[1].zeta_rot = 3
    assert bench.algorithmic_bytes(sp, counts, 1, b_v=8) == 10 * 2 * 25 + 5 * 2 * 39 + 64
    assert bench.algorithmic_bytes(sp, counts, 1, b_v=8, spatial=True) == 2 * (10 * 2 * 49 + 5 * 2 * 63) + 64


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_measured_traffic_is_tied_to_the_kernel_sources(monkeypatch, tmp_path):
    shape = {"block": 128, "group_slots": 2048}
    rec = tmp_path / "traffic.txt"
    rec.write_text(f"# header\ntraffic digest={bench.kernel_digest()} workload=chemistry-67m form=mixed "
                   "steps_per_launch=50 block=128 group_slots=2048 fetch_bytes=2e11 write_bytes=1e11\n")
    monkeypatch.setattr(bench, "TRAFFIC_PATH", str(rec))
    assert bench.measured_traffic("chemistry-67m", "mixed", shape) == pytest.approx(3e11 / 50)
    assert bench.measured_traffic("chemistry-67m", "fp64", shape) is None
    assert bench.measured_traffic("methane-argon", "mixed", shape) is None
    assert bench.measured_traffic("chemistry-67m", "mixed", {"block": 64, "group_slots": 2048}) is None
    monkeypatch.setattr(bench, "kernel_digest", lambda: "0" * 16)
    assert bench.measured_traffic("chemistry-67m", "mixed", shape) is None


@pytest.mark.parametrize("name", bench.WORKLOADS)
def test_every_workload_builds_and_has_a_tuned_shape(name):
    wl, desc = bench.make_workload(name)
    assert wl.n_cells > 0 and desc
    assert name in bench.TUNED_SHAPE
    if name.startswith("box"):
        assert wl.domain is not None and wl.domain[0] * wl.domain[1] * wl.domain[2] == wl.n_cells
    if name == "box-inflow-67m":
        assert wl.inflow is not None and wl.inflow[0] == 0b000011


def test_cpu_baseline_reports_the_oracle_on_a_bounded_sample():
    cb = bench.cpu_baseline("methane-argon", target_s=1.0)
    assert cb["kind"] == "oracle" and cb["cores"] == bench.host_threads() and cb["unit"] == "collisions/s"
    assert cb["value"] > 0 and "cells" in cb["sample"] and cb["cpu_model"]
    assert cb["single_thread"]["cores"] == 1 and cb["single_thread"]["value"] > 0


def test_oracle_threads_do_not_change_the_result():
    import numpy as np
    import oracle
    from paper_2606_31548_amd import workloads as W
    wl = W.methane_chemistry(n_cells=16, per_cell=64, recombination=True, t=12000.0)
    outs = []
    for threads in (1, 4):
        o = oracle.from_workload(wl)
        o.set_threads(threads)
        o.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
        o.step(wl.dt, 5)
        outs.append((o.read_all(), o.counters()))
    (a, ca), (b, cb) = outs
    for x, y in zip(a, b):
        assert np.array_equal(np.asarray(x).view(np.uint8), np.asarray(y).view(np.uint8))
    assert np.array_equal(ca, cb)
