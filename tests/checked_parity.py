"""Runs the bounds-checked library (libhcao_checked.so, selected by the
HCAO_LIBRARY variable the caller sets) through the paths whose indices it
checks, each held bit for bit to the oracle: the 0D chemistry with births
and deaths, the exact sampler with rotors, uneven batched reservoirs, the
spatial mode with open faces and with cells on both sides of the re-bin's
staging limit, and the mixed form's step. Any index outside
its array makes a call fail with HCAO_EBOUNDS. Prints one line per case and
"checked ok" at the end; exits non-zero on the first failure.

Run by tests/test_gpu_checked.py in a process of its own (one library per
process)."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

from paper_2606_31548_amd import hcao, workloads as W  # noqa: E402
import oracle  # noqa: E402
from test_gpu_parity import _compare_state  # noqa: E402


def pair(wl, steps, what, precision=None, positions=False):
    print(f"case: {what}", flush=True)
    o = oracle.from_workload(wl)
    g = hcao.from_workload(wl) if precision is None else hcao.from_workload(wl, precision=precision)
    o.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    g.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    for n in steps:
        o.step(wl.dt, n)
        g.step(wl.dt, n)
        g.sync()
        if precision is None:
            _compare_state(o, g, what)
            if positions:
                a = np.concatenate([o.read_pos(c) for c in range(o.n_cells)])
                assert np.array_equal(a.view(np.uint64), g.read_positions().view(np.uint64)), what
    counters = g.cell_state()[2].sum(0)
    o.close()
    g.close()
    return counters


def main():
    lib = os.path.basename(hcao.LIB_PATH)
    assert lib == "libhcao_checked.so", f"expected the bounds-checked library, got {lib}"
    hcao.load_library()
    oracle.build(force=False)

    # three-body recombination driven hard (n = 3e26 m^-3): deaths, compaction
    # and products within one step
    wl = W.methane_chemistry(n_cells=24, per_cell=256, recombination=True, t=6000.0)
    wl.cell_weight = wl.cell_weight * 3e4
    wl.dt = 5e-14
    ctr = pair(wl, (1, 29), "dense chemistry with recombination")
    assert ctr[hcao.CTR_BIRTHS] > 0 and ctr[hcao.CTR_DEATHS] > 0, ctr[:8]

    wl = W.methane_chemistry(n_cells=8, per_cell=256, recombination=True, t=12000.0)
    for s in wl.species:
        if s.n_modes:
            s.sampler = W.SAMPLER_EXACT
        if s.name in ("CH4", "CH3", "H2"):
            s.zeta_rot = 2 if s.name == "H2" else 3
    for r in wl.reactions:
        if r.kind != W.RX_RECOMBINATION:
            r.gamma_rot = 0.5
    pair(wl, (10,), "exact sampler and rotors")

    wl = W.batched_reservoirs(n_res=48, lo=20, hi=3000, seed=3)
    pair(wl, (4, 6), "uneven batched reservoirs")

    wl = W.spatial_box(nx=4, ny=3, nz=3, per_cell=150, chemistry=True, t_trans=12000.0, dt=5e-9,
                       open_faces=0b000011)
    pair(wl, (2, 10), "spatial chemistry with open faces", positions=True)

    # cells above the re-bin's LDS staging limit beside cells below it
    wl = W.spatial_box(nx=3, ny=2, nz=2, per_cell=150, periodic=0b111, t_trans=30000.0)
    wl.counts = wl.counts.copy()
    wl.counts[::3] *= 5
    wl.counts[1::3] *= 2
    wl.capacity_per_cell = 2048
    pair(wl, (1, 4), "spatial cells above and below the staging limit", positions=True)

    wl = W.methane_chemistry(n_cells=24, per_cell=256, recombination=True, t=12000.0)
    pair(wl, (20,), "mixed form", precision=hcao.MIXED)
    print("checked ok", flush=True)


if __name__ == "__main__":
    main()
