"""Benchmark of the HCAO DSMC collision step on one MI355X.

Workload (default): 262,144 reservoir cells x 256 particles (67.1M) of the
CH4/CH3/H/H2 chemistry (64 of each per cell, n = 1e22 m^-3, T 8,000 K,
dissociation CH4 + M -> CH3 + H + M, exchange CH4 + H -> CH3 + H2 and
recombination CH3 + H + M -> CH4 + M, dt 5e-9 s), synthetic thermal initial
state generated on the GPU. The mixed fp32/fp64 form is the headline value;
the fp64 form is timed beside it on the same workload, and both report the
energy drift over their run.

A step is one pass of the whole collision step over every cell (NTC
selection, VHS acceptance, reaction decision and application, relaxation,
scattering, product placement). The timed region covers exactly --steps
steps with the state resident in HBM, bracketed by stream synchronisation.

Prints one JSON line with the metric (collisions/s), the roofline of the
step kernel (algorithmic bytes per launch / mean launch duration from HIP
events recorded on the library's stream) and the CPU oracle (fp64) timed on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2606_31548_amd import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
TRAFFIC_PATH = os.path.join(ROOT, "profiles", "k_step_traffic.txt")


def algorithmic_bytes(wl_species, counts_by_species, n_cells, b_v=8, spatial=False):
    """Bytes one step must read and write: every live particle's velocity
    (3 b_v), species byte, 2-byte quantum number per mode it has and, for a
    rotor, 8-byte rotational energy, read and written once, plus 64 B of
    per-cell state. In the spatial mode each particle also carries a 24-byte
    position and its whole state is read and written a second time by the
    move and re-bin."""
    per = np.array([2 * (3 * b_v + 1 + 2 * s.n_modes + (8 if getattr(s, "zeta_rot", 0) else 0) +
                         (24 if spatial else 0)) for s in wl_species], np.float64)
    if spatial:
        per = 2 * per
    return float((counts_by_species * per).sum() + 64.0 * n_cells)


WORKLOADS = ("chemistry-67m", "chemistry-16m", "methane-argon", "batched", "triatomic", "box-67m",
             "box-inflow-67m")

# Launch shape (workgroup size, slot target per workgroup) per workload,
# the fastest over the timed steps in sweeps of block 64/128/256 and slot
# targets on MI355X; fixed here so that a profiled run holds only the timed
# launches. A slot target counts cell capacities: on the chemistry
# workloads (352 slots per cell) 2560 gives workgroups of seven cells, 3%
# (mixed) and 4% (fp64) faster than eight (2816 to 3072) and 2% faster than
# six; the spatial box (576 per cell) does best with six (3456), 2% faster
# than five or eight.
# --autotune runs the library's autotuner instead, after the warm-up.
TUNED_SHAPE = {"chemistry-67m": (128, 2560), "chemistry-16m": (128, 2560), "methane-argon": (64, 1024),
               "batched": (256, 4096), "triatomic": (64, 1024), "box-67m": (128, 3456),
               "box-inflow-67m": (128, 3456)}
# the batched leg of the default run, per form: 512-lane workgroups suit the
# fp64 form's large reservoirs (4.8 against 5.0 ms per step) and not the
# mixed form's (6.8 against 4.5)
BATCHED_LEG_SHAPE = {"mixed": (256, 4096), "fp64": (512, 8192)}


def make_workload(name):
    if name == "chemistry-67m":
        wl = W.methane_chemistry(n_cells=262144, per_cell=256, recombination=True)
        desc = ("262144 cells x 256 particles (67.1M), CH4/CH3/H/H2 64 each per cell, T 8000 K, "
                "dissociation + exchange + recombination, dt 5e-9 s")
    elif name == "chemistry-16m":
        wl = W.methane_chemistry(n_cells=65536, per_cell=256, recombination=True)
        desc = ("65536 cells x 256 particles (16.8M), CH4/CH3/H/H2 64 each per cell, T 8000 K, "
                "dissociation + exchange + recombination, dt 5e-9 s")
    elif name == "methane-argon":
        wl = W.methane_argon(n_cells=4096, per_cell=256)
        desc = "4096 cells x 256 particles, CH4-like/Ar-like 1:9, T_trans 20000 K, T_vib 300 K, " \
               "CH4+M->CH3+H+M, dt 1e-8 s"
    elif name == "batched":
        wl = W.batched_reservoirs(n_res=4096)
        desc = ("4096 independent reservoirs of the CH4-like/Ar-like 1:9 chemistry, particle counts log-uniform "
                f"in [1000, 100000] ({int(wl.n_particles)} in total), T_trans uniform in [5000, 30000] K, "
                "T_vib 300 K, CH4+M->CH3+H+M, dt 1e-8 s")
    elif name == "box-67m":
        wl = W.spatial_box(nx=64, ny=64, nz=64, per_cell=256, periodic=0b111, chemistry=True, t_trans=8000.0,
                           dt=5e-9)
        desc = ("spatial box of 64 x 64 x 64 cells of 0.1 mm (periodic), 256 particles per cell (67.1M), "
                "CH4/CH3/H/H2 64 each, T 8000 K, dissociation + exchange + recombination, dt 5e-9 s; every step "
                "moves, re-bins and collides")
    elif name == "box-inflow-67m":
        wl = W.spatial_box(nx=64, ny=64, nz=64, per_cell=256, periodic=0b110, chemistry=True, t_trans=8000.0,
                           dt=5e-9, open_faces=0b000011)
        desc = ("spatial channel of 64 x 64 x 64 cells of 0.1 mm, faces x = 0 and x = L open to a reservoir of the "
                "initial state (y, z periodic), 256 particles per cell (67.1M), CH4/CH3/H/H2 64 each, T 8000 K, "
                "dissociation + exchange + recombination, dt 5e-9 s; every step moves (particles leave through "
                "the open faces), admits the faces' inflow, re-bins and collides")
    elif name == "triatomic":
        wl = W.triatomic_reservoir(10000)
        desc = "1 cell x 10000 particles, synthetic triatomic, T_trans 10000 K, T_vib 300 K, dissociation"
    else:
        raise SystemExit(f"unknown workload {name}")
    return wl, desc


SAMPLERS = {"auto": W.SAMPLER_AUTO, "joint": W.SAMPLER_JOINT, "gibbs": W.SAMPLER_GIBBS, "exact": W.SAMPLER_EXACT}
SAMPLER_DESC = {"auto": "joint for 2-4 modes, Gibbs sweep otherwise", "joint": "joint proposal as printed",
                "gibbs": "Gibbs sweep", "exact": "exact joint sampler (per-mode Boltzmann proposals)"}


def recombination_exact(hcao, oracle_nodes=3):
    """Eq. recomb-correct for CH4 (9 modes, D_e 4.5 eV) over the 1024-node
    temperature table on the device, and the oracle's serial sum at a few of
    the nodes for comparison (time per temperature, largest relative
    difference)."""
    import oracle
    oracle.build(force=False)
    wl = W.methane_chemistry(n_cells=2, per_cell=16, recombination=True)
    g = hcao.from_workload(wl)
    nodes = np.exp(np.log(100.0) + np.arange(1024) * np.log(5e4 / 100.0) / 1023)
    g.recombination_exact(W.CH4, 4.5 * W.EV, 0.74, nodes[:4])  # warm-up
    p, ms, nrec = g.recombination_exact(W.CH4, 4.5 * W.EV, 0.74, nodes)
    o = oracle.from_workload(wl)
    worst, t0 = 0.0, time.perf_counter()
    for i in np.linspace(256, 1023, oracle_nodes).astype(int):
        want = o.rec_exact_probability(W.CH4, 4.5 * W.EV, 0.74, nodes[i])
        worst = max(worst, abs(p[i] / want - 1.0))
    cpu_per_t = (time.perf_counter() - t0) / oracle_nodes
    g.close()
    return {"species": "CH4 (9 modes)", "temperatures": 1024, "records": int(nrec), "device_ms": ms,
            "records_x_temperatures_per_s": nrec * 1024 / (ms * 1e-3),
            "oracle_s_per_temperature": cpu_per_t, "oracle_s_for_table": cpu_per_t * 1024,
            "max_rel_diff_vs_oracle": worst}


def set_rotors(wl, gamma=0.5):
    """Rotors on every molecule (zeta 3 for polyatomics, 2 for diatomics),
    rotation coupled into dissociation and exchange with gamma."""
    for s in wl.species:
        if s.n_modes:
            s.zeta_rot = 2 if s.n_modes == 1 else 3
    for r in wl.reactions:
        if r.kind != W.RX_RECOMBINATION:
            r.gamma_rot = gamma


def set_sampler(wl, sampler):
    for s in wl.species:
        if s.n_modes:
            s.sampler = SAMPLERS[sampler]


def host_threads():
    """Threads the host gives this process (affinity, capped by OMP_NUM_THREADS)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS", n)))
    except ValueError:
        pass
    return max(1, n)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, target_s=15.0, sampler="auto", rotors=False):
    """The oracle as it stands on a bounded sample of the same workload, on
    one thread and on all threads the host gives this process (threads over
    cells; the oracle's result does not depend on the count). The headline
    value is the all-threads leg."""
    threads = host_threads()
    one = _cpu_leg(name, 0.5 * target_s, sampler, rotors, 1)
    many = _cpu_leg(name, 0.5 * target_s, sampler, rotors, threads) if threads > 1 else one
    out = dict(many)
    out["cpu_model"] = cpu_model()
    out["single_thread"] = {k: one[k] for k in ("value", "cores", "sample")}
    return out


def _cpu_leg(name, target_s, sampler, rotors, threads):
    """One leg: a subset of the cells (for the spatial box an 8 x 8 x 8 box
    of the same cells), stepped from the same kind of initial state, until
    about target_s seconds of wall time are done."""
    import oracle
    oracle.build(force=False)
    wl, _ = make_workload(name)
    n_cells = min(wl.n_cells, 512)
    if getattr(wl, "domain", None) is not None:
        sub = W.spatial_box(nx=8, ny=8, nz=8, per_cell=256, periodic=wl.domain[6], chemistry=True,
                            t_trans=float(wl.t_trans[0]), dt=wl.dt,
                            open_faces=wl.inflow[0] if getattr(wl, "inflow", None) is not None else 0)
    else:
        sub = W.Workload(wl.name, wl.species, wl.reactions, wl.counts[:n_cells].copy(),
                         wl.t_trans[:n_cells].copy(), wl.t_vib[:n_cells].copy(), wl.cell_volume[:n_cells].copy(),
                         wl.cell_weight[:n_cells].copy(), dt=wl.dt, seed=wl.seed)
    set_sampler(sub, sampler)
    if rotors:
        set_rotors(sub)
    o = oracle.from_workload(sub)
    o.set_threads(threads)
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
    what = (f"an 8 x 8 x 8 box of the same cells (the workload has {wl.n_cells})"
            if getattr(wl, "domain", None) is not None else f"{n_cells} of {wl.n_cells} cells of the same workload")
    return {"value": coll / dt, "unit": "collisions/s", "cores": threads, "kind": "oracle",
            "sample": f"{what}, {steps} steps after 2 warm-up steps, {dt:.1f} s, "
                      f"{threads} thread{'s' if threads > 1 else ''} over cells"}


def kernel_digest():
    """Digest of the step kernel's sources: measured traffic is used only
    while the kernel it was measured on is unchanged."""
    import hashlib
    h = hashlib.sha256()
    for f in ("hcao_kernels.hip", "hcao_tables.h"):
        with open(os.path.join(ROOT, "paper_2606_31548_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, form, shape):
    """HBM bytes per step of the k_step launches from the rocprofv3
    FETCH_SIZE / WRITE_SIZE runs recorded in profiles/k_step_traffic.txt
    (lines 'traffic key=value ...', bytes per launch of steps_per_launch
    steps), or None when no record matches this kernel, workload, form and
    launch shape."""
    path = TRAFFIC_PATH
    if not os.path.exists(path):
        return None
    digest = kernel_digest()
    with open(path) as fh:
        for line in fh:
            if not line.startswith("traffic "):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            if (kv.get("digest") == digest and kv.get("workload") == workload and kv.get("form") == form
                    and int(kv.get("block", -1)) == shape["block"]
                    and int(kv.get("group_slots", -1)) == shape["group_slots"]):
                return (float(kv["fetch_bytes"]) + float(kv["write_bytes"])) / int(kv["steps_per_launch"])
    return None


def _energy(sim, m, n_modes):
    """Kinetic + vibrational (zero point included) + formation energy of the
    particles [J] and the thermal part (kinetic + vibrational above the zero
    point) that drift is measured against."""
    e = m.E_kin_J + m.E_formation_J
    th = m.E_kin_J
    for s in range(len(n_modes)):
        e += m.E_vib_J[s] + m.n_species[s] * sim.zero_point(s) + m.E_rot_J[s]
        th += m.E_vib_J[s] + m.E_rot_J[s]
    return e, th


def measure(hcao, torch, wl, precision, steps, warmup, spl, graph=False, autotune=False, shape=None,
            phase_clocks=False):
    """Times `steps` steps of one form after `warmup` untimed ones, every
    step-kernel launch advancing up to `spl` steps (the last launch of a
    call takes the remainder); returns throughput, the step kernel's roofline
    figures and the energy drift. graph: steps through the captured hipGraph
    form (one graph of spl steps per replay, and a remainder graph);
    autotune: picks the launch shape first; phase_clocks: per-phase clock
    shares of the timed steps (instrumented library only)."""
    stream = torch.cuda.Stream()
    sim = hcao.from_workload(wl, stream=hcao.ctypes.c_void_p(stream.cuda_stream), precision=precision)
    sim.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    if shape is None:
        cur = sim.launch_shape()  # defaults, or HCAO_BLOCK / HCAO_GROUP_SLOTS from the environment
        shape = (cur["block"], cur["group_slots"])
    sim.set_launch_shape(shape[0], shape[1], spl)
    n_modes = [sp.n_modes for sp in wl.species]
    m_init = sim.moments()
    e_init, th_init = _energy(sim, m_init, n_modes)
    # graph form: one captured graph of `chunk` steps, chunk dividing both
    # step counts, so that it is captured in the warm-up and only replayed
    # in the timed region
    chunk = math.gcd(math.gcd(spl, steps), warmup) if warmup else math.gcd(spl, steps)

    def advance(n):
        if not graph:
            sim.step(wl.dt, n)
            return
        for _ in range(n // chunk):
            sim.step_graph(wl.dt, chunk)
    advance(warmup)
    sim.sync()
    if autotune:
        # trials from the warmed state (the autotuner restores it afterwards)
        tuned = sim.autotune(wl.dt, trial_steps=min(spl, 20))
        sim.set_launch_shape(tuned["block"], tuned["group_slots"], spl)

    open_faces = getattr(wl, "inflow", None) is not None
    flux0 = sim.flux_counts()
    _, _, ctr0 = sim.cell_state()
    tot0 = sim.moments()
    per_species0 = np.array(tot0.n_species[:len(wl.species)], np.float64)
    if phase_clocks:
        sim.phase_clocks(reset=True)
    sim.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    advance(steps)
    sim.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms, launches, kernel_steps = sim.kernel_time()
    sim.set_timing(False)
    clocks = sim.phase_clocks() if phase_clocks else None
    _, _, ctr1 = sim.cell_state()
    tot1 = sim.moments()
    flux1 = sim.flux_counts()
    per_species1 = np.array(tot1.n_species[:len(wl.species)], np.float64)
    e_end, _ = _energy(sim, tot1, n_modes)

    coll = int(ctr1[:, hcao.CTR_COLLISIONS].sum() - ctr0[:, hcao.CTR_COLLISIONS].sum())
    cand = int(ctr1[:, hcao.CTR_CANDIDATES].sum() - ctr0[:, hcao.CTR_CANDIDATES].sum())
    trials = int(ctr1[:, hcao.CTR_TRIALS].sum() - ctr0[:, hcao.CTR_TRIALS].sum())
    reactions = int(ctr1[:, hcao.CTR_REACTION0:].sum() - ctr0[:, hcao.CTR_REACTION0:].sum())
    n_mean = 0.5 * (tot0.n_total + tot1.n_total)
    # algorithmic bytes per launch: per step, every live particle's state read
    # and written once plus 64 B per cell; a launch advances kernel_steps/launches steps
    b_v = 4 if precision == hcao.MIXED else 8
    spatial = getattr(wl, "domain", None) is not None
    b_step = 0.5 * (algorithmic_bytes(wl.species, per_species0, wl.n_cells, b_v, spatial) +
                    algorithmic_bytes(wl.species, per_species1, wl.n_cells, b_v, spatial))
    steps_per_launch = kernel_steps / max(launches, 1)
    b_alg = b_step * steps_per_launch
    avg_launch_s = kernel_ms / 1e3 / max(launches, 1)
    achieved = b_alg / avg_launch_s / 1e9
    r = {
        "collisions_per_s": coll / elapsed,
        "ms_per_step": elapsed * 1e3 / steps,
        "particle_steps_per_s": n_mean * steps / elapsed,
        "candidates": cand,
        "collisions": coll,
        "reactions": reactions,
        "sampler_trials_per_collision": trials / max(coll, 1),
        # relative to the initial thermal energy, over all warm-up and timed
        # steps (null with open faces: energy enters and leaves with particles)
        "energy_drift": None if open_faces else abs(e_end - e_init) / th_init,
        "energy_owed_rel": tot1.E_defect_J / th_init,
        "T_trans_K": tot1.T_trans_K,
        "launch_shape": dict(sim.launch_shape(), graph=graph, autotuned=autotune),
        # particles admitted through and gone out of open faces in the timed steps
        "flux": {"admitted": flux1[0] - flux0[0], "left": flux1[1] - flux0[1]} if open_faces else None,
        "phase_clock_shares": phase_shares(clocks) if clocks else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_step", "bytes_per_launch": b_alg, "steps_per_launch": steps_per_launch,
                     "mean_launch_us": avg_launch_s * 1e6},
    }
    sim.close()
    return r


def phase_shares(clocks):
    """Shares of the step kernel's phases (workgroup clocks) and, separately,
    of the collision phase's parts (wave clocks)."""
    step = {k: v for k, v in clocks.items() if not k.startswith("collide_")}
    parts = {k: v for k, v in clocks.items() if k.startswith("collide_")}
    out = {k: v / max(sum(step.values()), 1) for k, v in step.items()}
    out.update({k: v / max(sum(parts.values()), 1) for k, v in parts.items()})
    return out


def precision_report(hcao, torch, wl, steps=10000, spl=50):
    """Both forms run `steps` untimed steps from the same thermal initial
    state: energy drift of each (relative to the initial thermal energy),
    and per observable the two forms' values with the statistical error of
    each (cells are independent replicas of the reservoir, so the error of a
    per-cell mean is the cells' spread over sqrt(cells); a total's is the
    spread times sqrt(cells)), the relative error of mixed against fp64 and
    their difference in units of the combined sigma. Observables: the
    translational temperature and each molecular species' vibrational
    temperature (per-cell means), particles per cell of each species, and
    reactions per channel over the run."""
    n_modes = [sp.n_modes for sp in wl.species]
    forms = {}
    for name, prec in (("mixed", hcao.MIXED), ("fp64", hcao.FP64)):
        print(f"# precision report: {steps} steps of the {name} form", file=sys.stderr, flush=True)
        sim = hcao.from_workload(wl, precision=prec)
        sim.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
        sim.set_launch_shape(*TUNED_SHAPE.get(getattr(wl, "bench_name", ""), (128, 3072)), spl)
        m0 = sim.moments()
        e0, th0 = _energy(sim, m0, n_modes)
        t0 = time.perf_counter()
        sim.step(wl.dt, steps)
        sim.sync()
        wall = time.perf_counter() - t0
        m1 = sim.moments()
        e1, _ = _energy(sim, m1, n_modes)
        per = sim.moments_per_cell()
        ctr = sim.cell_state()[2]
        nc = len(per)
        obs = {}

        def mean_of(x, name):
            x = np.asarray(x, np.float64)
            obs[name] = (float(x.mean()), float(x.std(ddof=1) / np.sqrt(len(x))))

        mean_of(per["T_trans_K"], "T_trans_K")
        for s, sp in enumerate(wl.species):
            mean_of(per["n_species"][:, s], f"n_per_cell[{sp.name}]")
            if sp.n_modes:
                have = per["n_species"][:, s] > 0
                if have.sum() > 1:
                    mean_of(per["T_vib_K"][have, s], f"T_vib_K[{sp.name}]")
        for r in range(len(wl.reactions)):
            x = ctr[:, hcao.CTR_REACTION0 + r].astype(np.float64)
            obs[f"reactions[{r}]"] = (float(x.sum()), float(x.std(ddof=1) * np.sqrt(nc)))
        forms[name] = {"energy_drift": abs(e1 - e0) / th0, "energy_owed_rel": m1.E_defect_J / th0,
                       "steps": steps, "wall_s": wall, "observables": obs}
        sim.close()
    comp = {}
    for k, (vm, sm) in forms["mixed"]["observables"].items():
        if k not in forms["fp64"]["observables"]:
            continue
        vf, sf = forms["fp64"]["observables"][k]
        sig = float(np.hypot(sm, sf))
        comp[k] = {"mixed": vm, "fp64": vf, "sigma_mixed": sm, "sigma_fp64": sf,
                   "rel_err": (vm - vf) / vf if vf else None,
                   "z": abs(vm - vf) / sig if sig > 0 else (0.0 if vm == vf else float("inf"))}
    return {"steps": steps, "cells": wl.n_cells, "particles": int(wl.n_particles),
            "energy_drift": {f: forms[f]["energy_drift"] for f in forms},
            "energy_owed_rel_mixed": forms["mixed"]["energy_owed_rel"],
            "wall_s": {f: forms[f]["wall_s"] for f in forms},
            "mixed_vs_fp64": comp,
            "max_z": max((c["z"] for c in comp.values()), default=0.0),
            "mixed_drift_within_1e-6": forms["mixed"]["energy_drift"] <= 1e-6}


def copy_peak(torch, mib=1024, repeats=10):
    """HBM bandwidth that a plain device-to-device copy reaches (bytes read
    plus bytes written per second, HIP events around `repeats` copies of
    `mib` MiB): the practical ceiling beside the datasheet's 8 TB/s."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(repeats):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbs = 2 * n * 8 * repeats / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def measure_sequential(hcao, torch, wl, steps):
    """The same reservoirs run one at a time: one context and one launch per
    reservoir and step (what the batched launch replaces)."""
    stream = torch.cuda.Stream()
    sims = []
    for r in range(wl.n_cells):
        one = W.Workload(wl.name, wl.species, wl.reactions, wl.counts[r:r + 1].copy(), wl.t_trans[r:r + 1].copy(),
                         wl.t_vib[r:r + 1].copy(), wl.cell_volume[r:r + 1].copy(), wl.cell_weight[r:r + 1].copy(),
                         dt=wl.dt, seed=wl.seed + r)
        s = hcao.from_workload(one, stream=hcao.ctypes.c_void_p(stream.cuda_stream))
        s.init_thermal(one.counts, one.t_trans, one.t_vib)
        sims.append(s)
    for s in sims:
        s.step(wl.dt, 1)
    torch.cuda.synchronize()
    c0 = sum(int(s.cell_state()[2][:, hcao.CTR_COLLISIONS].sum()) for s in sims)
    t0 = time.perf_counter()
    for _ in range(steps):
        for s in sims:
            s.step(wl.dt, 1)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    c1 = sum(int(s.cell_state()[2][:, hcao.CTR_COLLISIONS].sum()) for s in sims)
    for s in sims:
        s.close()
    return {"collisions_per_s": (c1 - c0) / elapsed, "ms_per_step": elapsed * 1e3 / steps, "steps": steps,
            "launches_per_step": wl.n_cells}


def batched_leg(hcao, torch, steps):
    """The batched-reservoir workload beside the headline: its mixed and fp64
    forms through the captured graph at the tuned launch shape (steps timed
    after as many warm-up steps), their energy drift, and the same reservoirs
    stepped one launch per reservoir (fp64, two steps)."""
    wl, desc = make_workload("batched")
    wl.bench_name = "batched"
    spl = math.gcd(steps, 50)
    out = {"workload": desc, "cells": wl.n_cells, "particles": int(wl.n_particles), "steps": steps,
           "warmup": steps}
    for f in ("mixed", "fp64"):
        print(f"# batched reservoirs, {f} form: {steps} warm-up + {steps} steps", file=sys.stderr, flush=True)
        shape = BATCHED_LEG_SHAPE[f]
        r = measure(hcao, torch, wl, hcao.MIXED if f == "mixed" else hcao.FP64, steps, steps, spl, graph=True,
                    shape=shape)
        out[f] = {k: r[k] for k in ("collisions_per_s", "particle_steps_per_s", "ms_per_step", "energy_drift",
                                    "T_trans_K", "reactions")}
        out[f]["launch_shape"] = {"block": shape[0], "group_slots": shape[1], "steps_per_launch": spl}
    out["mixed_vs_fp64"] = out["mixed"]["collisions_per_s"] / out["fp64"]["collisions_per_s"]
    print("# batched reservoirs, one launch per reservoir (fp64)", file=sys.stderr, flush=True)
    seq = measure_sequential(hcao, torch, wl, 2)
    out["sequential_fp64"] = seq
    out["batched_vs_sequential_fp64"] = out["fp64"]["collisions_per_s"] / seq["collisions_per_s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--steps-per-launch", type=int, default=50,
                    help="steps per step-kernel launch (the last launch of the warm-up or of the timed region "
                         "takes the remainder)")
    ap.add_argument("--workload", default="chemistry-67m", choices=WORKLOADS)
    ap.add_argument("--precision", default="both", choices=("both", "mixed", "fp64"),
                    help="both: the mixed form is the headline value, the fp64 form is timed beside it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="run the library's autotuner before timing (default for the batched workload)")
    ap.add_argument("--library-shape", action="store_true",
                    help="use the library's default launch shape (or HCAO_BLOCK / HCAO_GROUP_SLOTS) instead of "
                         "the tuned one")
    ap.add_argument("--sampler", default="auto", choices=SAMPLERS,
                    help="relaxation sampler of every molecular species")
    ap.add_argument("--rotors", action="store_true",
                    help="give every molecule a rotor and couple rotation into its reactions (gamma 0.5)")
    ap.add_argument("--recomb-exact", action="store_true",
                    help="also time Eq. recomb-correct for CH4 on the device against the oracle")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--batched-steps", type=int, default=50,
                    help="chemistry workloads: steps of the batched-reservoir leg (mixed and fp64, captured "
                         "graph, after as many warm-up steps) reported beside the headline; 0 skips it")
    ap.add_argument("--precision-steps", type=int, default=10000,
                    help="steps of the untimed precision report (both forms from the same initial state: energy "
                         "drift, temperatures, species and reaction counts of mixed against fp64); 0 skips it")
    ap.add_argument("--phase-clocks", action="store_true",
                    help="report per-phase clock shares of the step kernel (needs the instrumented library: "
                         "python paper_2606_31548_amd/build.py --phase-clocks, then HCAO_LIBRARY="
                         "paper_2606_31548_amd/libhcao_clocks.so)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a device-to-device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path (asked for --gpus {args.gpus})",
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
    wl.bench_name = args.workload
    set_sampler(wl, args.sampler)
    if args.rotors:
        set_rotors(wl)
        desc += "; every molecule a rotor, rotation coupling 0.5"
    spl = max(1, args.steps_per_launch)
    steps = args.steps
    warmup = max(0, args.warmup)
    if steps < 1:
        print("bench.py needs --steps >= 1", file=sys.stderr)
        sys.exit(2)
    forms = {"both": ("mixed", "fp64"), "mixed": ("mixed",), "fp64": ("fp64",)}[args.precision]
    batched = args.workload == "batched"
    res = {}
    for f in forms:
        print(f"# timing the {f} form: {warmup} warm-up + {steps} steps, up to {spl} per launch",
              file=sys.stderr, flush=True)
        res[f] = measure(hcao, torch, wl, hcao.MIXED if f == "mixed" else hcao.FP64, steps, warmup, spl,
                         graph=batched, autotune=args.autotune or batched,
                         shape=None if args.library_shape else TUNED_SHAPE[args.workload],
                         phase_clocks=args.phase_clocks)
        per_step = (measured_traffic(args.workload, f, res[f]["launch_shape"])
                    if args.sampler == "auto" and not args.rotors else None)
        res[f]["roofline"]["traffic"] = (per_step * res[f]["roofline"]["steps_per_launch"]
                                         if per_step is not None else None)
    cp = copy_peak(torch)
    for f in res:
        res[f]["roofline"]["frac_of_copy"] = res[f]["roofline"]["achieved"] / cp
    head = res[forms[0]]
    out = {
        "metric": "HCAO collisions/s on 1 MI355X; mixed FP32/FP64 vs FP64 at fixed energy error",
        "value": head["collisions_per_s"],
        "unit": "collisions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if forms[0] == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "cells": wl.n_cells, "particles": int(wl.n_particles),
                   "precision": forms[0], "sampler": SAMPLER_DESC[args.sampler]},
        "particle_steps_per_s": head["particle_steps_per_s"],
        "energy_drift": head["energy_drift"],
        "roofline": head["roofline"],
        # a 1 GiB device-to-device copy, bytes read plus written per second
        "copy_peak_GBs": cp,
        "forms": res,
    }
    if "mixed" in res and "fp64" in res:
        out["mixed_vs_fp64"] = res["mixed"]["collisions_per_s"] / res["fp64"]["collisions_per_s"]
    if batched:
        print("# timing per-reservoir sequential launches (fp64)", file=sys.stderr, flush=True)
        seq = measure_sequential(hcao, torch, wl, 2)
        out["sequential_fp64"] = seq
        if "fp64" in res:
            out["batched_vs_sequential_fp64"] = res["fp64"]["collisions_per_s"] / seq["collisions_per_s"]
    if args.batched_steps > 0 and args.workload in ("chemistry-67m", "chemistry-16m"):
        out["batched"] = batched_leg(hcao, torch, args.batched_steps)
    if args.precision_steps > 0 and args.workload in ("chemistry-67m", "chemistry-16m"):
        out["precision_report"] = precision_report(hcao, torch, wl, args.precision_steps, spl)
    if args.recomb_exact:
        print("# Eq. recomb-correct for CH4 on the device and in the oracle", file=sys.stderr, flush=True)
        out["recombination_exact"] = recombination_exact(hcao)
    if not args.no_cpu_baseline:
        print("# timing the oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds, args.sampler, args.rotors)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
