"""Benchmark of the HCAO DSMC collision step on one MI355X.

Workload (default): 4,096 reservoir cells x 256 particles (1,048,576),
methane-like molecules (16 amu, 4 Morse C-H stretches, 5 bends) in an
argon-like bath at 1:9, T_trans 20,000 K, T_vib 300 K, dissociation
CH4 + M -> CH3 + H + M, fp64, dt 1e-8 s; synthetic thermal initial state
generated on the GPU.

A step is one pass of the whole collision step over every cell (NTC
selection, VHS acceptance, reaction decision and application, relaxation,
scattering, product placement). The timed region covers exactly --steps
steps with the state resident in HBM, bracketed by stream synchronisation.

Prints one JSON line with the metric (collisions/s), the roofline of the
step kernel (algorithmic bytes per launch / mean launch duration from HIP
events recorded on the library's stream) and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2606_31548_amd import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(wl_species, counts_by_species, n_cells, b_v=8):
    """Bytes one step must read and write: every live particle's velocity
    (3 b_v), species byte and 2-byte quantum number per mode it has, read and
    written once, plus 64 B of per-cell state."""
    per = np.array([2 * (3 * b_v + 1 + 2 * s.n_modes) for s in wl_species], np.float64)
    return float((counts_by_species * per).sum() + 64.0 * n_cells)


def make_workload(name):
    if name == "methane-argon":
        wl = W.methane_argon(n_cells=4096, per_cell=256)
        desc = "4096 cells x 256 particles, CH4-like/Ar-like 1:9, T_trans 20000 K, T_vib 300 K, " \
               "CH4+M->CH3+H+M, fp64, dt 1e-8 s"
    elif name == "methane-chemistry":
        wl = W.methane_chemistry(n_cells=65536, per_cell=256, recombination=False)
        desc = "65536 cells x 256 particles, CH4/CH3/H/H2, T 8000 K, dissociation + exchange, fp64, dt 1e-8 s"
    elif name == "triatomic":
        wl = W.triatomic_reservoir(10000)
        desc = "1 cell x 10000 particles, synthetic triatomic, T_trans 10000 K, T_vib 300 K, dissociation, fp64"
    else:
        raise SystemExit(f"unknown workload {name}")
    return wl, desc


def cpu_baseline(name, target_s=15.0):
    """The oracle as it stands (single thread) on a bounded sample of the
    same workload: a subset of the cells, stepped from the same kind of
    initial state, until about target_s seconds of CPU work are done."""
    import oracle
    oracle.build(force=False)
    wl, _ = make_workload(name)
    n_cells = min(wl.n_cells, 512)
    sub = W.Workload(wl.name, wl.species, wl.reactions, wl.counts[:n_cells].copy(), wl.t_trans[:n_cells].copy(),
                     wl.t_vib[:n_cells].copy(), wl.cell_volume[:n_cells].copy(), wl.cell_weight[:n_cells].copy(),
                     dt=wl.dt, seed=wl.seed)
    o = oracle.from_workload(sub)
    o.init_thermal(sub.counts, sub.t_trans, sub.t_vib)
    o.step(sub.dt, 2)  # warm-up
    c0 = o.counters()[:, oracle.CTR_COLLISIONS].sum()
    steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < target_s:
        o.step(sub.dt, 5)
        steps += 5
    dt = time.perf_counter() - t0
    coll = int(o.counters()[:, oracle.CTR_COLLISIONS].sum() - c0)
    return {"value": coll / dt, "unit": "collisions/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_cells} of {wl.n_cells} cells of the same workload, {steps} steps after 2 warm-up "
                      f"steps, {dt:.1f} s, single thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="methane-argon")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device-to-device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_31548_amd import hcao

    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.rand(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "repeats": 5}))
        return

    wl, desc = make_workload(args.workload)
    stream = torch.cuda.Stream()
    sim = hcao.from_workload(wl, stream=hcao.ctypes.c_void_p(stream.cuda_stream))
    sim.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    sim.step(wl.dt, args.warmup)
    sim.sync()

    _, _, ctr0 = sim.cell_state()
    tot0 = sim.moments()
    per_species0 = np.array(tot0.n_species[:len(wl.species)], np.float64)
    sim.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(wl.dt, args.steps)
    sim.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms, launches, kernel_steps = sim.kernel_time()
    sim.set_timing(False)
    _, _, ctr1 = sim.cell_state()
    tot1 = sim.moments()
    per_species1 = np.array(tot1.n_species[:len(wl.species)], np.float64)

    coll = int(ctr1[:, hcao.CTR_COLLISIONS].sum() - ctr0[:, hcao.CTR_COLLISIONS].sum())
    cand = int(ctr1[:, hcao.CTR_CANDIDATES].sum() - ctr0[:, hcao.CTR_CANDIDATES].sum())
    trials = int(ctr1[:, hcao.CTR_TRIALS].sum() - ctr0[:, hcao.CTR_TRIALS].sum())
    reactions = int(ctr1[:, hcao.CTR_REACTION0:].sum() - ctr0[:, hcao.CTR_REACTION0:].sum())
    n_mean = 0.5 * (tot0.n_total + tot1.n_total)
    # algorithmic bytes per launch: per step, every live particle's state read
    # and written once plus 64 B per cell; a launch advances kernel_steps/launches steps
    b_step = 0.5 * (algorithmic_bytes(wl.species, per_species0, wl.n_cells) +
                    algorithmic_bytes(wl.species, per_species1, wl.n_cells))
    steps_per_launch = kernel_steps / max(launches, 1)
    b_alg = b_step * steps_per_launch
    avg_launch_s = kernel_ms / 1e3 / max(launches, 1)
    achieved = b_alg / avg_launch_s / 1e9

    out = {
        "metric": "HCAO collisions/s on 1 MI355X",
        "value": coll / elapsed,
        "unit": "collisions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "cells": wl.n_cells, "particles": int(wl.n_particles), "precision": "fp64",
                   "sampler": "joint <= 4 modes, Gibbs sweep otherwise"},
        "particle_steps_per_s": n_mean * args.steps / elapsed,
        "candidates": cand,
        "collisions": coll,
        "reactions": reactions,
        "sampler_trials_per_collision": trials / max(coll, 1),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_step", "bytes_per_launch": b_alg, "steps_per_launch": steps_per_launch,
                     "mean_launch_us": avg_launch_s * 1e6},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
