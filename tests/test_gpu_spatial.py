"""Spatial mode on the GPU: ballistic movement with periodic and specular
walls, the per-step stable re-bin (a device radix sort of the particles
that left their cell), then the collision step,
against the fp64 oracle bit for bit (positions, velocities, cell order,
species, levels, counters)."""
import numpy as np
import pytest

from paper_2606_31548_amd import workloads as W
from test_gpu_parity import _compare_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    from paper_2606_31548_amd import hcao
    hcao.load_library()
    return hcao


def _compare_pos(o, g, what):
    a = np.concatenate([o.read_pos(c) for c in range(o.n_cells)])
    b = g.read_positions()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), f"{what}: positions differ"


@pytest.mark.parametrize("periodic", [0b000, 0b111, 0b011])
def test_spatial_step_parity(orc, hc, periodic):
    """Methane/argon at 30,000 K in a 6 x 5 x 4 box of 0.1 mm cells: a
    particle crosses about half a cell per step, so the re-bin moves many
    particles every step; dissociation births inherit positions."""
    wl = W.spatial_box(nx=6, ny=5, nz=4, per_cell=200, periodic=periodic, t_trans=30000.0)
    o = orc.from_workload(wl)
    g = hc.from_workload(wl)
    o.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    g.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    _compare_state(o, g, "init")
    _compare_pos(o, g, "init")
    counts0 = np.array([o.count(c) for c in range(wl.n_cells)])
    done = 0
    for n in (1, 9, 20):
        o.step(wl.dt, n)
        g.step(wl.dt, n)
        g.sync()
        done += n
        _compare_state(o, g, f"after {done} steps")
        _compare_pos(o, g, f"after {done} steps")
    counts1 = np.array([o.count(c) for c in range(wl.n_cells)])
    assert np.any(counts0 != counts1)
    assert o.counters().sum(0)[orc.CTR_REACTION0] > 0


def test_spatial_chemistry_with_rotors_parity(orc, hc):
    """The CH4/CH3/H/H2 chemistry (recombination included) with rotors in a
    periodic box, from a loaded state with given positions."""
    wl = W.spatial_box(nx=4, ny=4, nz=3, per_cell=200, periodic=0b111, chemistry=True, t_trans=12000.0, dt=5e-9)
    for s in wl.species:
        if s.name in ("CH4", "CH3", "H2"):
            s.zeta_rot = 2 if s.name == "H2" else 3
    for r in wl.reactions:
        if r.kind != W.RX_RECOMBINATION:
            r.gamma_rot = 0.5
    cell, sp, v, lv = W.random_state(wl, seed=31)
    nx, ny, nz, lx, ly, lz, _ = wl.domain
    rng = np.random.default_rng(31)
    ijk = np.stack([cell % nx, (cell // nx) % ny, cell // (nx * ny)], 1)
    d = np.array([lx / nx, ly / ny, lz / nz])
    pos = (ijk + rng.random((len(cell), 3)) * 0.999) * d
    rot = np.where(np.isin(sp, [W.CH4, W.CH3, W.H2]), rng.gamma(1.5, W.K_BOLTZ * 12000.0, len(sp)), 0.0)
    o = orc.from_workload(wl)
    g = hc.from_workload(wl)
    o.load(cell, sp, v, lv, rot, pos)
    g.load_particles(cell, sp, v, lv, rot, pos)
    for n in (5, 15):
        o.step(wl.dt, n)
        g.step(wl.dt, n)
        g.sync()
        _compare_state(o, g, "chemistry box")
        _compare_pos(o, g, "chemistry box")
    a = np.concatenate([o.read_rot(c) for c in range(o.n_cells)])
    assert np.array_equal(a.view(np.uint64), g.read_rotational_energy().view(np.uint64))


def test_spatial_mode_refusals_and_checkpoint(hc, tmp_path):
    wl = W.spatial_box(nx=3, ny=3, nz=3, per_cell=100, periodic=0b111)
    g = hc.from_workload(wl)
    g.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    with pytest.raises(hc.HcaoError):
        g.step_graph(wl.dt, 2)
    cell, sp, v, lv = W.random_state(wl, seed=3)
    with pytest.raises(hc.HcaoError):
        g.load_particles(cell, sp, v, lv)  # no positions
    bad = np.zeros((len(cell), 3))  # every particle at the origin: not in its cell
    with pytest.raises(hc.HcaoError):
        g.load_particles(cell, sp, v, lv, None, bad)
    a = hc.from_workload(wl)
    a.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    a.step(wl.dt, 20)
    b = hc.from_workload(wl)
    b.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    b.step(wl.dt, 10)
    b.save(tmp_path / "box.bin")
    c = hc.from_workload(wl)
    c.restore(tmp_path / "box.bin")
    c.step(wl.dt, 10)
    for x, y in zip(a.read_particles(), c.read_particles()):
        assert np.array_equal(np.asarray(x).view(np.uint8), np.asarray(y).view(np.uint8))
    assert np.array_equal(a.read_positions().view(np.uint64), c.read_positions().view(np.uint64))


def test_spatial_mixed_form_conserves_energy(hc):
    wl = W.spatial_box(nx=6, ny=6, nz=6, per_cell=200, periodic=0b000, t_trans=30000.0)
    g = hc.from_workload(wl, precision=hc.MIXED)
    g.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    m0 = g.moments()
    e0 = g.total_energy(m0)
    scale = m0.E_kin_J + sum(m0.E_vib_J[s] for s in range(g.n_species))
    g.step(wl.dt, 200)
    g.sync()
    m1 = g.moments()
    assert abs(g.total_energy(m1) - e0) / scale < 1e-11
    pos = g.read_positions()
    nx, ny, nz, lx, ly, lz, _ = wl.domain
    assert np.all(pos >= 0) and np.all(pos <= np.array([lx, ly, lz]))


def test_spatial_parity_with_multi_chunk_scans(orc, hc):
    """A 16 x 16 x 8 box (2,048 cells, 540k slots): the re-bin's radix sort
    scans digit histograms of several scan chunks."""
    wl = W.spatial_box(nx=16, ny=16, nz=8, per_cell=100, periodic=0b101, t_trans=25000.0)
    o = orc.from_workload(wl)
    g = hc.from_workload(wl)
    o.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    g.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    for n in (1, 3):
        o.step(wl.dt, n)
        g.step(wl.dt, n)
        g.sync()
        _compare_state(o, g, "multi-chunk box")
        _compare_pos(o, g, "multi-chunk box")


def test_spatial_rebin_capacity_overflow_is_reported(orc, hc):
    """Two cells of capacity 150: the 100 particles of cell 0 all fly into
    cell 1, which already holds 100. The re-bin drops nothing silently: both
    the oracle and the library report a capacity error."""
    sp = [W.Species("Ar", 40 * W.AMU)]
    edge = 1e-4
    wl = W.Workload("overflow", sp, [], np.array([[100], [100]]), np.full(2, 300.0), np.full(2, 300.0),
                    np.full(2, edge ** 3), np.full(2, 1e-30), dt=1e-8, capacity_per_cell=150,
                    domain=(2, 1, 1, 2 * edge, edge, edge, 0))
    rng = np.random.default_rng(9)
    cell = np.repeat(np.arange(2, dtype=np.uint32), 100)
    pos = np.stack([(cell + 0.25 + 0.5 * rng.random(200)) * edge, rng.random(200) * edge,
                    rng.random(200) * edge], 1)
    vel = np.zeros((200, 3))
    vel[:100, 0] = 0.9 * edge / wl.dt  # crosses into cell 1 within one step, stays clear of the far wall
    o = orc.from_workload(wl)
    g = hc.from_workload(wl)
    o.load(cell, np.zeros(200, np.uint8), vel, np.zeros((200, 1), np.uint16), None, pos)
    g.load_particles(cell, np.zeros(200, np.uint8), vel, np.zeros((200, 1), np.uint16), None, pos)
    with pytest.raises(orc.OracleError):
        o.step(wl.dt, 1)
    with pytest.raises(hc.HcaoError):
        g.step(wl.dt, 1)
        g.sync()


def test_spatial_rebin_large_and_small_cells_parity(orc, hc):
    """Cells of 750, 300 and 150 particles side by side in a periodic box:
    the place pass stages a cell's fields through LDS only up to 384 old
    slots (up to 256 in one register set per thread, beyond that in a
    second), so movers flow between cells that take the staged path with
    one or two slots per thread and cells that copy directly."""
    wl = W.spatial_box(nx=3, ny=2, nz=2, per_cell=150, periodic=0b111, t_trans=30000.0)
    wl.counts = wl.counts.copy()
    wl.counts[::3] *= 5
    wl.counts[1::3] *= 2
    wl.capacity_per_cell = 2048
    o = orc.from_workload(wl)
    g = hc.from_workload(wl)
    o.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    g.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    sizes = [o.count(c) for c in range(wl.n_cells)]
    assert max(sizes) > 384 and any(256 < n <= 384 for n in sizes) and min(sizes) <= 256
    for n in (1, 5):
        o.step(wl.dt, n)
        g.step(wl.dt, n)
        g.sync()
        _compare_state(o, g, f"large and small cells: {n} steps")
        _compare_pos(o, g, f"large and small cells: {n} steps")


@pytest.mark.parametrize("shape,dt", [((3, 3, 2), 1e-13), ((1, 2, 5), None)])
def test_spatial_rebin_without_movers_and_on_thin_axes(orc, hc, shape, dt):
    """The re-bin sorts only the particles that leave their cell. A step
    too short for anyone to leave takes the path with no movers; a periodic
    box one and two cells thick wraps movers onto their own cell's
    neighbours from both sides."""
    nx, ny, nz = shape
    wl = W.spatial_box(nx=nx, ny=ny, nz=nz, per_cell=150, periodic=0b111, t_trans=30000.0)
    if dt is not None:
        wl.dt = dt
    o = orc.from_workload(wl)
    g = hc.from_workload(wl)
    o.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    g.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    before = np.array([o.count(c) for c in range(wl.n_cells)])
    for n in (1, 6):
        o.step(wl.dt, n)
        g.step(wl.dt, n)
        g.sync()
        _compare_state(o, g, f"{shape}: {n} steps")
        _compare_pos(o, g, f"{shape}: {n} steps")
    after = np.array([o.count(c) for c in range(wl.n_cells)])
    if dt is None:
        assert np.any(before != after)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_spatial_launch_shape_invariance(hc, monkeypatch, precision):
    """Movement, re-bin and collisions give the same bits for every launch
    shape (workgroup size, slots per workgroup), in both forms."""
    wl = W.spatial_box(nx=8, ny=6, nz=5, per_cell=180, periodic=0b101, chemistry=True, t_trans=12000.0, dt=5e-9)
    prec = hc.FP64 if precision == "fp64" else hc.MIXED
    outs = []
    for block, slots in (("64", "1"), ("128", "3072"), ("256", "4608")):
        monkeypatch.setenv("HCAO_BLOCK", block)
        monkeypatch.setenv("HCAO_GROUP_SLOTS", slots)
        g = hc.from_workload(wl, precision=prec)
        g.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
        g.step(wl.dt, 15)
        g.sync()
        outs.append((g.read_particles(), g.read_positions(), g.cell_state()[2]))
        g.close()
    for parts, pos, ctr in outs[1:]:
        for a, b in zip(outs[0][0], parts):
            assert np.array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8))
        assert np.array_equal(outs[0][1].view(np.uint64), pos.view(np.uint64))
        assert np.array_equal(outs[0][2], ctr)
    assert outs[0][2][:, 1].sum() > 0
