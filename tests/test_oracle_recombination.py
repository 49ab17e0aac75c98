"""Pins of the oracle's recombination model (Sec. "Recombination reactions"):
the regularized upper incomplete gamma against closed forms and scipy, the
Whitten-Rabinovich density of states (one oscillator, branch continuity at
the zero-point energy, high-energy limit), vibrational partition sums,
per-collision recombination frequency, conservation in recombining
collisions and atom bookkeeping over a reservoir run."""
import math

import numpy as np
import pytest
from scipy import special, stats

from paper_2606_31548_amd import workloads as W

KB, H, EV = W.K_BOLTZ, W.H_PLANCK, W.EV


def test_incomplete_gamma_closed_forms(orc):
    for x in (1e-6, 0.1, 0.9, 1.0, 2.5, 7.0, 30.0, 200.0):
        assert abs(orc.gamma_q(1.0, x) / math.exp(-x) - 1) < 1e-13
        assert abs(orc.gamma_q(0.5, x) / math.erfc(math.sqrt(x)) - 1) < 1e-12
    assert orc.gamma_q(1.76, 0.0) == 1.0 and orc.gamma_q(1.76, -3.0) == 1.0


def test_incomplete_gamma_matches_scipy(orc):
    rng = np.random.default_rng(3)
    for a, x in zip(rng.uniform(0.3, 3.0, 400), np.exp(rng.uniform(-6, 5, 400))):
        want = special.gammaincc(a, x)
        got = orc.gamma_q(a, x)
        assert abs(got - want) <= 1e-13 + 1e-11 * want


def _build(orc, species, reactions=()):
    o = orc.Oracle(1, 1, W.VOLUME, 1e10)
    for s in species:
        o.add_species(s)
    for r in reactions:
        o.add_reaction(r)
    o.finalize()
    return o


def test_wr_density_single_oscillator_is_constant(orc):
    """With l = 1 the Whitten-Rabinovich expression is 1/(h nu) at every energy."""
    theta = 1500.0
    o = _build(orc, [W.Species("X", 20 * W.AMU, bend_theta_K=[theta])])
    hnu = KB * theta
    for e in (0.0, 0.01 * EV, 0.3 * EV, 3.0 * EV):
        assert abs(o.wr_rho(0, e) * hnu - 1) < 1e-12


def test_wr_density_branches_meet_at_zero_point(orc):
    """The two branches of Omega meet at E = E_z only with a base-10 log:
    10^-1.0506 = 0.0890 = 1/(5 + 2.73 + 3.51)."""
    sp = W.methane_species()
    o = _build(orc, sp)
    nus = [KB * t / H for t in sp[0].bend_theta_K]
    for m in range(5, 9):
        lev = o.levels(0, m)
        nus.append((lev[1] - lev[0]) / H)
    ez = 0.5 * H * sum(nus)
    lo, hi = o.wr_rho(0, ez * (1 - 1e-12)), o.wr_rho(0, ez * (1 + 1e-12))
    assert abs(hi / lo - 1) < 5e-4
    # high energy: a(E) -> 1, rho -> (E + E_z)^(l-1) / ((l-1)! prod h nu)
    e = 200 * ez
    want = (e + ez) ** 8 / (math.factorial(8) * np.prod([H * x for x in nus]))
    assert abs(o.wr_rho(0, e) / want - 1) < 1e-3


def test_vibrational_partition_sums(orc):
    sp = W.methane_species()
    o = _build(orc, sp)
    for t in (500.0, 4000.0, 20000.0):
        want = 1.0
        for th in sp[0].bend_theta_K:
            want /= (1 - math.exp(-th / t))
        for m in range(5, 9):
            lev = o.levels(0, m)
            want *= float(np.exp(-(lev - lev[0]) / (KB * t)).sum())
        assert abs(o.q_vib(0, t) / want - 1) < 1e-12
    assert o.q_vib(1, 3000.0) == 1.0  # atom


def test_wr_probability_tracks_exact_level_sum(orc):
    """Eq. recomb-correct (sum over all level combinations) against its
    Whitten-Rabinovich approximation for a 2-stretch, 1-bend molecule. The
    paper only says the deviation is small: parity unpinned, a factor-2
    sanity band."""
    sp = W.triatomic_species()
    o = _build(orc, sp)
    lev = [o.levels(0, 0, 200), o.levels(0, 1), o.levels(0, 2)]
    de = 5.5 * EV
    a = 2.5 - 0.74
    for t in (6000.0, 10000.0, 20000.0):
        e = (lev[0][:, None, None] - lev[0][0]) + (lev[1][None, :, None] - lev[1][0]) + \
            (lev[2][None, None, :] - lev[2][0])
        w = np.exp(-e / (KB * t))
        g = special.gammaincc(a, np.maximum(de - e, 0) / (KB * t))
        exact = float((g * w).sum() / w.sum())
        approx = o.wr_probability(0, de, 0.74, 1000, t)
        assert 0.5 < approx / exact < 2.0, (t, approx, exact)


@pytest.mark.parametrize("t", [1500.0, 3000.0, 6000.0, 10000.0, 20000.0])
def test_exact_recombination_sum_matches_box_enumeration(orc, t):
    """Eq. recomb-correct by the oracle's depth-first walk (closed-form tails
    above D_e) against a brute-force sum over a level box of the triatomic
    (bend truncated at 900 levels, far above D_e), down to P ~ 1e-15."""
    sp = W.triatomic_species()
    o = _build(orc, sp)
    lev = [o.levels(0, 0, 900), o.levels(0, 1), o.levels(0, 2)]
    de = 5.5 * EV
    a = 2.5 - 0.74
    e = (lev[0][:, None, None] - lev[0][0]) + (lev[1][None, :, None] - lev[1][0]) + \
        (lev[2][None, None, :] - lev[2][0])
    w = np.exp(-e / (KB * t))
    g = special.gammaincc(a, np.maximum(de - e, 0) / (KB * t))
    box = float((g * w).sum() / w.sum())
    got = o.rec_exact_probability(0, de, 0.74, t)
    assert abs(got / box - 1) < 1e-12, (got, box)


def test_exact_recombination_single_oscillator_closed_form(orc):
    """One harmonic oscillator of spacing eps and a = 1 (Q(1, x) = e^-x): the
    J levels below D contribute e^(-D/kT) each, the rest their Boltzmann
    weight, so P = (1 - r) (J e^(-D/kT) + r^J / (1 - r)), r = e^(-eps/kT)."""
    theta = 1800.0
    o = _build(orc, [W.Species("osc", 20 * W.AMU, bend_theta_K=[theta])])
    eps = KB * theta
    for de_ev, t in ((0.9, 700.0), (2.0, 3000.0), (5.0, 12000.0), (3.1, 40000.0)):
        de = de_ev * EV
        j = math.ceil(de / eps)
        r = math.exp(-eps / (KB * t))
        want = (1 - r) * (j * math.exp(-de / (KB * t)) + r ** j / (1 - r))
        got = o.rec_exact_probability(0, de, 1.5, t)
        assert abs(got / want - 1) < 1e-12, (de_ev, t, got, want)


def _recomb_setup(orc):
    sp = W.methane_species()
    rx = [W.methane_dissociation(), W.methane_exchange(), W.methyl_recombination()]
    return sp, _build(orc, sp, rx)


def test_recombination_frequency_matches_probability(orc):
    """CH3 + H with an Ar third body at fixed cell temperature and density:
    the fraction that recombines is min(1, k_b n / <sigma g>_BC)."""
    sp, o = _recomb_setup(orc)
    n = 20000
    t_cell = 4000.0
    for target in (0.3, 0.7):
        n_cell = target / o.rec_factor(2, W.AR, t_cell)
        pr = min(1.0, o.rec_factor(2, W.AR, t_cell) * n_cell)
        rng = np.random.default_rng(int(target * 100))
        pairs = np.tile([W.CH3, W.H], n)
        masses = np.array([s.mass_kg for s in sp])[pairs]
        vel = rng.standard_normal((2 * n, 3)) * np.sqrt(KB * t_cell / masses)[:, None]
        lvl = np.zeros((2 * n, o.max_modes), np.uint16)
        m_sp = np.full(n, W.AR, np.uint8)
        m_vel = rng.standard_normal((n, 3)) * math.sqrt(KB * t_cell / sp[W.AR].mass_kg)
        sp_o, vel_o, lvl_o, rxo, m_vel_o = o.collide3_batch(pairs, vel, lvl, m_sp, m_vel, t_cell, n_cell)
        frac = (rxo == 2).mean()
        assert 0.01 < pr < 0.99
        assert abs(frac - pr) < 4 * math.sqrt(pr * (1 - pr) / n)


def test_recombining_collisions_conserve_energy_and_momentum(orc):
    sp, o = _recomb_setup(orc)
    n = 3000
    rng = np.random.default_rng(9)
    pairs = np.tile([W.H, W.CH3], n)
    masses = np.array([s.mass_kg for s in sp])
    vel = rng.standard_normal((2 * n, 3)) * np.sqrt(KB * 6000.0 / masses[pairs])[:, None]
    lvl = np.zeros((2 * n, o.max_modes), np.uint16)
    lvl[1::2, :3] = rng.integers(0, 3, size=(n, 3))
    m_sp = rng.choice([W.AR, W.CH4, W.H2], size=n).astype(np.uint8)
    m_vel = rng.standard_normal((n, 3)) * np.sqrt(KB * 6000.0 / masses[m_sp])[:, None]
    sp_o, vel_o, lvl_o, rxo, m_vel_o = o.collide3_batch(pairs, vel, lvl, m_sp, m_vel, 6000.0, 1e32)
    rec = rxo == 2
    assert rec.sum() > 100

    def energy(s, v, l):
        e = 0.5 * masses[s] * (v * v).sum(-1) + np.array([x.formation_J for x in sp])[s]
        for i in range(len(s)):
            _, nm, _ = o.species_info(int(s[i]))
            for m in range(nm):
                e[i] += o.levels(int(s[i]), m, int(l[i, m]) + 1)[int(l[i, m])]
        return e

    e0 = energy(pairs, vel, lvl).reshape(n, 2).sum(1) + energy(m_sp, m_vel, np.zeros((n, o.max_modes), int))
    alive = sp_o != 255
    s1 = np.where(alive, sp_o, 0)
    e1 = np.where(alive, energy(s1, vel_o, lvl_o), 0.0).reshape(n, 2).sum(1) + \
        energy(m_sp, m_vel_o, np.zeros((n, o.max_modes), int))
    scale = 0.5 * (masses[pairs] * (vel * vel).sum(-1)).reshape(n, 2).sum(1) + 5 * EV
    assert np.all(np.abs(e1 - e0) <= 1e-12 * scale)
    p0 = (masses[pairs][:, None] * vel).reshape(n, 2, 3).sum(1) + masses[m_sp][:, None] * m_vel
    p1 = (np.where(alive, masses[s1], 0.0)[:, None] * vel_o).reshape(n, 2, 3).sum(1) + masses[m_sp][:, None] * m_vel_o
    pscale = np.abs(p0).sum(1) + 1e-30
    assert np.all(np.abs(p1 - p0).max(1) <= 1e-12 * pscale)
    # the recombined pair: one CH4 and one removed particle
    assert np.all(np.sort(sp_o.reshape(n, 2)[rec], axis=1) == [W.CH4, 255])


def test_reservoir_with_recombination_keeps_atoms(orc):
    """A dense CH4/CH3/H/H2 reservoir with all three reactions: carbon and
    hydrogen atoms are conserved, the count change equals births - deaths."""
    wl = W.methane_chemistry(n_cells=6, per_cell=256, recombination=True, t=6000.0)
    wl.cell_weight = wl.cell_weight * 1e5  # n = 1e27 m^-3: frequent three-body events
    wl.dt = 5e-14
    o = orc.from_workload(wl)
    o.init_thermal(wl.counts, wl.t_trans, wl.t_vib)
    c_atoms = np.array([1, 0, 1, 0, 0])
    h_atoms = np.array([4, 0, 3, 1, 2])

    def atoms():
        _, s, _, _ = o.read_all()
        return c_atoms[s].sum(), h_atoms[s].sum(), len(s)

    a0 = atoms()
    o.step(wl.dt, 40)
    a1 = atoms()
    ctr = o.counters().sum(0)
    assert a1[:2] == a0[:2]
    assert a1[2] - a0[2] == int(ctr[orc.CTR_BIRTHS]) - int(ctr[orc.CTR_DEATHS])
    assert ctr[orc.CTR_REACTION0 + 2] == ctr[orc.CTR_DEATHS] > 0
