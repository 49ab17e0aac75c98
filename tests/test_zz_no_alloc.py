"""The allocation-free step (hcao_step_static) against the ordinary step
(hcao_step), through the C ABI: bitwise the same particles, cell state and
counters, on two calls in a row whose second context is smaller (the fixed
device array keeps the first call's contents), in both precisions, with the
exact sampler and rotors (the products staging of rotational energy); and
the refusals, decided on the host before anything runs: a context whose
scratch exceeds the fixed array, and the spatial mode."""
import numpy as np
import pytest

from paper_2606_31548_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    from paper_2606_31548_amd import hcao
    hcao.load_library()
    return hcao


def _same(a, b, what):
    ac, asp, av, al = a.read_particles()
    bc, bsp, bv, bl = b.read_particles()
    assert np.array_equal(ac, bc), f"{what}: per-cell counts differ"
    assert np.array_equal(asp, bsp), f"{what}: species differ"
    assert np.array_equal(al, bl), f"{what}: quantum numbers differ"
    assert np.array_equal(av.view(np.uint64), bv.view(np.uint64)), f"{what}: velocities differ"
    for x, y in zip(a.cell_state(), b.cell_state()):
        assert np.array_equal(np.asarray(x).view(np.uint8), np.asarray(y).view(np.uint8)), f"{what}: cell state"
    if a.precision == 1:
        ea, eb = a.moments().E_defect_J, b.moments().E_defect_J
        assert np.float64(ea).view(np.uint64) == np.float64(eb).view(np.uint64), f"{what}: energy owed"


def _pair(hc, wl, precision, rotors=False):
    out = []
    for _ in range(2):
        s = hc.from_workload(wl, precision=precision)
        s.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
        out.append(s)
    return out


def _rotor_chemistry(n_cells, per_cell):
    wl = W.methane_chemistry(n_cells=n_cells, per_cell=per_cell, recombination=True, t=12000.0)
    for s in wl.species:
        if s.n_modes:
            s.zeta_rot = 2 if s.n_modes == 1 else 3
            s.sampler = W.SAMPLER_EXACT
    for r in wl.reactions:
        if r.kind != W.RX_RECOMBINATION:
            r.gamma_rot = 0.5
    return wl


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_static_step_equals_step_on_two_calls_second_smaller(hc, precision):
    for n_cells, per_cell in ((96, 256), (7, 100)):
        wl = W.methane_chemistry(n_cells=n_cells, per_cell=per_cell, recombination=True, t=12000.0)
        print(f"static step: {n_cells} x {per_cell}, precision {precision}", flush=True)
        a, b = _pair(hc, wl, precision)
        a.step(wl.dt, 12)
        b.step_static(wl.dt, 12)
        a.sync()
        b.sync()
        _same(a, b, f"{n_cells} x {per_cell}")
        a.close()
        b.close()


def test_static_step_with_exact_sampler_and_rotors(hc):
    wl = _rotor_chemistry(40, 256)
    for precision in (0, 1):
        print(f"static step with rotors, precision {precision}", flush=True)
        a, b = _pair(hc, wl, precision)
        a.step(wl.dt, 8)
        b.step_static(wl.dt, 8)
        a.sync()
        b.sync()
        _same(a, b, "rotors")
        ra, rb = a.read_rotational_energy(), b.read_rotational_energy()
        assert np.array_equal(ra.view(np.uint64), rb.view(np.uint64))
        a.close()
        b.close()


def test_static_step_refuses_a_context_beyond_the_fixed_array(hc):
    wl = W.methane_chemistry(n_cells=16384, per_cell=256, recombination=True)
    s = hc.from_workload(wl)
    s.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    before = s.read_particles()
    with pytest.raises(hc.HcaoError) as e:
        s.step_static(wl.dt, 1)
    assert e.value.code == -5 and "fixed device array" in str(e.value)
    assert s.step_index == 0
    after = s.read_particles()
    assert np.array_equal(before[3], after[3]) and np.array_equal(before[2].view(np.uint64), after[2].view(np.uint64))
    s.close()


def test_static_step_refuses_the_spatial_mode(hc):
    wl = W.spatial_box(nx=4, ny=4, nz=4, per_cell=64, periodic=0b111)
    s = hc.from_workload(wl)
    s.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    with pytest.raises(hc.HcaoError) as e:
        s.step_static(wl.dt, 1)
    assert e.value.code == -8
    s.close()
