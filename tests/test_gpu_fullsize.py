"""Parity at the workloads' full sizes, in the launch configuration bench.py
times (autotuned launch shape, 50 steps per launch).

Cells are independent and every random draw is keyed by the global cell
index, so the oracle runs only a sample of the cells (first, last, middle and
random ones) at their global indices, from the same thermal initial state,
and those cells must match the GPU bit for bit. The mixed form, which is not
bitwise the oracle's, is held at full size to properties that hold at any
size: its fp64 energy audit closes, and atoms are conserved by every
reaction."""
import numpy as np
import pytest

from paper_2606_31548_amd import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 50


@pytest.fixture(scope="module")
def hc():
    from paper_2606_31548_amd import hcao
    hcao.load_library()
    return hcao


def _sample(n_cells, seed, k=5):
    rng = np.random.default_rng(seed)
    return sorted({0, 1, n_cells // 2, n_cells - 1} | set(int(c) for c in rng.choice(n_cells, k, replace=False)))


def _gpu_bench_config(hc, wl, precision):
    g = hc.from_workload(wl, precision=precision)
    g.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    shape = g.launch_shape()
    g.set_launch_shape(shape["block"], shape["group_slots"], STEPS)
    shape = g.autotune(wl.dt, trial_steps=3)
    g.set_launch_shape(shape["block"], shape["group_slots"], STEPS)
    assert g.step_index == 0
    g.step(wl.dt, STEPS)
    g.sync()
    return g


def _sampled_parity(orc, hc, wl, seed):
    cells = _sample(wl.n_cells, seed)
    print(f"sampled cells {cells} of {wl.n_cells}", flush=True)
    g = _gpu_bench_config(hc, wl, hc.FP64)
    counts = np.zeros_like(wl.counts)
    counts[cells] = wl.counts[cells]
    o = orc.from_workload(wl)
    o.init_thermal(counts, wl.t_trans, wl.t_vib)
    o.step(wl.dt, STEPS)
    gsg, grem, gctr = g.cell_state()
    collided = 0
    for c in cells:
        osp, ov, ol = o.read_cell(c)
        gsp, gv, gl = g.read_cell(c)
        assert np.array_equal(osp, gsp), f"cell {c}: species differ"
        assert np.array_equal(ol, gl[:, :ol.shape[1]]), f"cell {c}: quantum numbers differ"
        assert np.array_equal(ov.view(np.uint64), gv.view(np.uint64)), f"cell {c}: velocities differ"
        sg, rem, ctr = o.cell_state(c)
        assert sg == gsg[c] and rem == grem[c], f"cell {c}: (sigma g)_max or remainder differ"
        assert np.array_equal(ctr, gctr[c]), f"cell {c}: counters differ"
        collided += int(ctr[orc.CTR_COLLISIONS])
    assert collided > 0
    return g, o, cells


def test_fullsize_precision_chemistry_sampled_cells(orc, hc):
    """262,144 cells x 256 (67.1 M particles), fp64 form."""
    _sampled_parity(orc, hc, W.methane_chemistry(n_cells=262144, per_cell=256, recombination=True), seed=1)


def test_fullsize_exact_sampler_sampled_cells(orc, hc):
    """262,144 cells x 256 with every molecule on the exact sampler of the
    joint relaxation target (bench.py --sampler exact), fp64 form."""
    wl = W.methane_chemistry(n_cells=262144, per_cell=256, recombination=True)
    for sp in wl.species:
        if sp.n_modes:
            sp.sampler = W.SAMPLER_EXACT
    _sampled_parity(orc, hc, wl, seed=4)


def test_fullsize_rotors_sampled_cells(orc, hc):
    """262,144 cells x 256 with every molecule a rotor and rotation coupled
    into dissociation and exchange with 0.5 (bench.py --rotors), fp64 form;
    rotational energies too."""
    wl = W.methane_chemistry(n_cells=262144, per_cell=256, recombination=True)
    for sp in wl.species:
        if sp.n_modes:
            sp.zeta_rot = 2 if sp.n_modes == 1 else 3
    for r in wl.reactions:
        if r.kind != W.RX_RECOMBINATION:
            r.gamma_rot = 0.5
    g, o, cells = _sampled_parity(orc, hc, wl, seed=5)
    per, _ = g.counts()
    start = np.concatenate([[0], np.cumsum(per.astype(np.int64))])
    rot = g.read_rotational_energy()
    for c in cells:
        assert np.array_equal(o.read_rot(c).view(np.uint64), rot[start[c]:start[c + 1]].view(np.uint64)), f"cell {c}"


def test_fullsize_methane_argon_sampled_cells(orc, hc):
    """4,096 cells x 256 (1.05 M particles)."""
    _sampled_parity(orc, hc, W.methane_argon(n_cells=4096, per_cell=256), seed=2)


def test_fullsize_batched_reservoirs_sampled_cells(orc, hc):
    """4,096 reservoirs of 1,000 .. 100,000 particles (88 M in total); the
    sample includes the largest reservoir."""
    wl = W.batched_reservoirs(n_res=4096)
    big = int(np.argmax(wl.counts.sum(1)))
    cells = _sample(wl.n_cells, 3, k=3) + [big]
    counts = np.zeros_like(wl.counts)
    counts[cells] = wl.counts[cells]
    g = _gpu_bench_config(hc, wl, hc.FP64)
    o = orc.from_workload(wl)
    o.init_thermal(counts, wl.t_trans, wl.t_vib)
    o.step(wl.dt, STEPS)
    gsg, grem, gctr = g.cell_state()
    for c in sorted(set(cells)):
        osp, ov, ol = o.read_cell(c)
        gsp, gv, gl = g.read_cell(c)
        assert np.array_equal(osp, gsp) and np.array_equal(ol, gl[:, :ol.shape[1]]), f"reservoir {c}"
        assert np.array_equal(ov.view(np.uint64), gv.view(np.uint64)), f"reservoir {c}"
        assert np.array_equal(o.cell_state(c)[2], gctr[c]), f"reservoir {c}"


def _atoms(m):
    # C and H atoms of CH4, Ar, CH3, H, H2
    n = np.array(m.n_species[:5], np.int64)
    return n[0] + n[2], 4 * n[0] + 3 * n[2] + n[3] + 2 * n[4]


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_fullsize_precision_chemistry_invariants(hc, precision):
    """262,144 cells x 256: the energy audit closes to fp64 rounding and C
    and H atoms are conserved, in the bench's launch configuration."""
    wl = W.methane_chemistry(n_cells=262144, per_cell=256, recombination=True)
    prec = hc.MIXED if precision == "mixed" else hc.FP64
    g = hc.from_workload(wl, precision=prec)
    g.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    m0 = g.moments()
    e0 = g.total_energy(m0)
    scale = m0.E_kin_J + sum(m0.E_vib_J[s] for s in range(g.n_species))
    shape = g.autotune(wl.dt, trial_steps=3)
    g.set_launch_shape(shape["block"], shape["group_slots"], STEPS)
    g.step(wl.dt, STEPS)
    g.sync()
    m1 = g.moments()
    assert abs(g.total_energy(m1) - e0) / scale < 1e-11
    assert abs(g.total_energy(m1, with_defect=False) - e0) / scale < 1e-6
    assert _atoms(m0) == _atoms(m1)
    assert g.reaction_counts().sum() > 0
