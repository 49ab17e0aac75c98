"""Synthetic workloads: species tables, reactions, compositions and seeded inputs.

This module holds data and seeded random inputs only (none of the collision
method's arithmetic), so that the GPU library and the CPU oracle can be fed
identical inputs. Species parameters follow the spectroscopic tables of the
paper's verification section (methane, methyl radical, molecular hydrogen)
and the synthetic species of the benchmark configurations.

Common readings for all workloads (the paper states no workload sizes for a
GPU run): total number density 1e22 m^-3 per cell, reservoir volume
4.64e-6 m^3 (verification section), particle weight F_N = n V / N, time step
1e-8 s, and VHS d_ref = 4.0e-10 m, omega = 0.74, T_ref = 273 K for every
species.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

# exact SI constants used for unit conversion of the input data
H_PLANCK = 6.62607015e-34
C_LIGHT = 299792458.0
K_BOLTZ = 1.380649e-23
AMU = 1.66053906660e-27
EV = 1.602176634e-19

SAMPLER_AUTO, SAMPLER_JOINT, SAMPLER_GIBBS, SAMPLER_EXACT = 0, 1, 2, 3
RX_DISSOCIATION, RX_EXCHANGE, RX_RECOMBINATION = 0, 1, 2
REC_WR, REC_EXACT = 0, 1

VOLUME = 4.64e-6
DENSITY = 1e22
DT = 1e-8
VHS = dict(dref_m=4.0e-10, omega=0.74, Tref_K=273.0)


def theta_from_wavenumber(cm_inv: float) -> float:
    """Characteristic temperature [K] of a harmonic mode given in cm^-1."""
    return H_PLANCK * C_LIGHT * (cm_inv * 100.0) / K_BOLTZ


@dataclass
class Species:
    name: str
    mass_kg: float
    bend_theta_K: Sequence[float] = ()
    omega_e_per_m: Sequence[float] = ()
    chi_e: Sequence[float] = ()
    De_J: Sequence[float] = ()
    levels_J: Optional[Sequence[Sequence[float]]] = None
    formation_J: float = 0.0
    p_vib: float = 1.0
    sampler: int = SAMPLER_AUTO
    zeta_rot: int = 0      # rotational degrees of freedom (0, 2 or 3)
    p_rot: float = 0.2     # rotational relaxation probability per collision
    coupling: float = 0.0
    dref_m: float = VHS["dref_m"]
    omega: float = VHS["omega"]
    Tref_K: float = VHS["Tref_K"]

    @property
    def n_modes(self) -> int:
        return len(self.bend_theta_K) + len(self.omega_e_per_m)


@dataclass
class Reaction:
    kind: int
    reactant: Sequence[int]
    product: Sequence[int]
    stretch_mask: int = 0
    alpha: Optional[Sequence[float]] = None
    steric: float = 1.0
    Ea_J: float = 0.0
    n_samp: int = 1000
    rec_model: int = REC_WR
    gamma_rot: float = 0.0  # degree of rotation coupling (dissociation, exchange)


@dataclass
class Workload:
    name: str
    species: List[Species]
    reactions: List[Reaction]
    counts: np.ndarray            # [n_cells, n_species] initial composition
    t_trans: np.ndarray           # [n_cells] K
    t_vib: np.ndarray             # [n_cells] K
    cell_volume: np.ndarray       # [n_cells] m^3
    cell_weight: np.ndarray       # [n_cells] F_N
    dt: float = DT
    steps: int = 1
    seed: int = 0
    capacity_per_cell: int = 0
    notes: str = ""
    domain: Optional[tuple] = None  # spatial mode: (nx, ny, nz, lx, ly, lz, periodic axis bits)
    # spatial mode, open faces: (face bits 2 axis + side, reservoir number
    # densities [n_species] m^-3, T_trans, T_vib)
    inflow: Optional[tuple] = None

    @property
    def n_cells(self) -> int:
        return int(self.counts.shape[0])

    @property
    def n_particles(self) -> int:
        return int(self.counts.sum())

    @property
    def max_modes(self) -> int:
        return max(s.n_modes for s in self.species)


# ---------------------------------------------------------------------------
# species
# ---------------------------------------------------------------------------

def triatomic_species():
    """Synthetic triatomic A (44 amu; 2 stretches 2300 cm^-1, x_e 0.006,
    D_e 5.5 eV; 1 bend 670 cm^-1), its diatomic fragment B (28 amu, one
    identical stretch) and atom C (16 amu). Formation energies: A -5.5 eV,
    fragments 0, so the bond enthalpy equals D_e."""
    we = 2300.0 * 100.0
    de = 5.5 * EV
    a = Species("A", 44 * AMU, bend_theta_K=[theta_from_wavenumber(670.0)], omega_e_per_m=[we, we],
                chi_e=[0.006, 0.006], De_J=[de, de], formation_J=-5.5 * EV, coupling=0.05)
    b = Species("B", 28 * AMU, omega_e_per_m=[we], chi_e=[0.006], De_J=[de])
    c = Species("C", 16 * AMU)
    return [a, b, c]


def methane_species():
    """Methane-like chemistry. CH4: 16 amu, 4 C-H stretches 3020 cm^-1, x_e
    0.021, D_e 4.5 eV; 5 bends (2 x 1530, 3 x 1310 cm^-1). CH3: 15 amu, 3
    stretches as CH4, bends 872.1 K and 2 x 2016.2 K (methyl table of the
    paper). Ar: 40 amu. H: 1 amu. H2: 2 amu, 439524 m^-1, x_e 0.0287 (paper),
    D_e 4.747 eV. Formation energies: CH4 -4.5 eV, H2 -4.747 eV, others 0."""
    we, xe, de = 3020.0 * 100.0, 0.021, 4.5 * EV
    t1530, t1310 = theta_from_wavenumber(1530.0), theta_from_wavenumber(1310.0)
    ch4 = Species("CH4", 16 * AMU, bend_theta_K=[t1530, t1530, t1310, t1310, t1310],
                  omega_e_per_m=[we] * 4, chi_e=[xe] * 4, De_J=[de] * 4, formation_J=-4.5 * EV)
    ar = Species("Ar", 40 * AMU)
    ch3 = Species("CH3", 15 * AMU, bend_theta_K=[872.1, 2016.2, 2016.2], omega_e_per_m=[we] * 3,
                  chi_e=[xe] * 3, De_J=[de] * 3)
    h = Species("H", 1 * AMU)
    h2 = Species("H2", 2 * AMU, omega_e_per_m=[439524.0], chi_e=[0.0287], De_J=[4.747 * EV],
                 formation_J=-4.747 * EV)
    return [ch4, ar, ch3, h, h2]


CH4, AR, CH3, H, H2 = range(5)


def methane_dissociation():
    return Reaction(RX_DISSOCIATION, (CH4, -1), (CH3, H), stretch_mask=0b1111)


def methane_exchange():
    """CH4 + H -> CH3 + H2, barrier 0.6 eV, alpha 0.21 on the four C-H
    stretches and 0 on the bends (mode-selective coupling)."""
    return Reaction(RX_EXCHANGE, (CH4, H), (CH3, H2), alpha=[0.0] * 5 + [0.21] * 4, steric=1.0, Ea_J=0.6 * EV)


def methyl_recombination():
    return Reaction(RX_RECOMBINATION, (CH3, H), (CH4, -1), stretch_mask=0b1111)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def _uniform_cells(n_cells, per_cell_counts, t_trans, t_vib, density=DENSITY, volume=VOLUME):
    counts = np.tile(np.asarray(per_cell_counts, np.int64), (n_cells, 1))
    n = counts.sum(axis=1).astype(np.float64)
    vol = np.full(n_cells, volume)
    wgt = density * vol / n
    return counts, np.full(n_cells, float(t_trans)), np.full(n_cells, float(t_vib)), vol, wgt


def triatomic_reservoir(n_particles=10_000, steps=1000, dissociation=True, seed=0, sampler=SAMPLER_AUTO):
    """1 cell of the synthetic triatomic: T_trans 10,000 K, T_vib 300 K."""
    sp = triatomic_species()
    sp[0].sampler = sampler
    rx = [Reaction(RX_DISSOCIATION, (0, -1), (1, 2), stretch_mask=0b11)] if dissociation else []
    counts, tt, tv, vol, wgt = _uniform_cells(1, [n_particles, 0, 0], 10_000.0, 300.0)
    return Workload("triatomic-1cell", sp, rx, counts, tt, tv, vol, wgt, steps=steps, seed=seed)


def methane_argon(n_cells=4096, per_cell=256, steps=2000, seed=0, t_trans=20_000.0, t_vib=300.0):
    """CH4-like / Ar-like 1:9 reservoir cells with CH4 + M -> CH3 + H + M."""
    n_ch4 = int(round(0.1 * per_cell))
    counts, tt, tv, vol, wgt = _uniform_cells(n_cells, [n_ch4, per_cell - n_ch4, 0, 0, 0], t_trans, t_vib)
    return Workload(f"ch4-ar-{n_cells}x{per_cell}", methane_species(), [methane_dissociation()], counts, tt, tv,
                    vol, wgt, steps=steps, seed=seed)


def methane_chemistry(n_cells=65_536, per_cell=256, steps=5000, seed=0, t=8000.0, recombination=True, dt=5e-9):
    """CH4/H/CH3/H2 at equal densities with dissociation, exchange and (optionally)
    recombination, T_trans = T_vib = 8000 K. Time step 5e-9 s, the paper's
    value for its methane/hydrogen reservoir at 1e22 m^-3: with light atoms
    the collision frequency per particle is ~0.3 per 1e-8 s, which would push
    the disjoint-pair candidate count to its N/2 ceiling."""
    q = per_cell // 4
    counts, tt, tv, vol, wgt = _uniform_cells(n_cells, [q, 0, q, q, per_cell - 3 * q], t, t)
    rx = [methane_dissociation(), methane_exchange()]
    if recombination:
        rx.append(methyl_recombination())
    return Workload(f"ch4-h-ch3-h2-{n_cells}x{per_cell}", methane_species(), rx, counts, tt, tv, vol, wgt,
                    dt=dt, steps=steps, seed=seed)


def batched_reservoirs(n_res=4096, lo=1_000, hi=100_000, seed=0, steps=1000):
    """Independent 0D reservoirs of the CH4/Ar chemistry with log-uniform
    particle counts in [lo, hi] and T_trans uniform in [5000, 30000] K."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0xB47C]))
    u = rng.random(n_res)
    n_r = np.floor(np.exp(np.log(lo) + u * np.log(hi / lo))).astype(np.int64)
    t_tr = 5000.0 + 25000.0 * rng.random(n_res)
    n_ch4 = np.rint(0.1 * n_r).astype(np.int64)
    counts = np.zeros((n_res, 5), np.int64)
    counts[:, CH4] = n_ch4
    counts[:, AR] = n_r - n_ch4
    vol = np.full(n_res, VOLUME)
    wgt = DENSITY * vol / n_r
    return Workload(f"batched-{n_res}", methane_species(), [methane_dissociation()], counts, t_tr,
                    np.full(n_res, 300.0), vol, wgt, steps=steps, seed=seed)


# ---------------------------------------------------------------------------
# seeded random particle states (for the host-array load path)
# ---------------------------------------------------------------------------

def spatial_box(nx=16, ny=16, nz=16, per_cell=256, cell_edge=1e-4, periodic=0, chemistry=False,
                t_trans=20_000.0, t_vib=300.0, dt=1e-8, seed=0, open_faces=0, empty=False):
    """A box of nx x ny x nz cubic cells of edge cell_edge [m] at density
    1e22 m^-3 (F_N = n V_cell / per_cell), walls specular except on the
    periodic axes (bits 0..2). Species and reactions of the methane/argon
    workload (or, with chemistry=True, the CH4/CH3/H/H2 chemistry at
    t_trans). A particle at 5 km/s crosses half a 0.1 mm cell per 1e-8 s
    step, so the per-step re-binning moves a large share of particles.
    Cells get room for twice their initial count. open_faces (bits 2 axis +
    side, on non-periodic axes) opens faces to a reservoir of the initial
    composition, density and temperatures; empty=True starts the box with
    no particles (it then fills through its open faces)."""
    n_cells = nx * ny * nz
    vol = cell_edge ** 3
    if chemistry:
        base = methane_chemistry(n_cells=n_cells, per_cell=per_cell, recombination=True, t=t_trans, dt=dt)
    else:
        base = methane_argon(n_cells=n_cells, per_cell=per_cell, t_trans=t_trans, t_vib=t_vib)
        base.dt = dt
    base.cell_volume = np.full(n_cells, vol)
    base.cell_weight = np.full(n_cells, DENSITY * vol / per_cell)
    base.domain = (nx, ny, nz, nx * cell_edge, ny * cell_edge, nz * cell_edge, periodic)
    # cells exchange particles every step and the chemistry adds products:
    # room for twice the initial count
    base.capacity_per_cell = 2 * per_cell + 64
    base.name = f"box-{nx}x{ny}x{nz}"
    base.seed = seed
    if open_faces:
        frac = base.counts[0] / float(per_cell)
        base.inflow = (open_faces, DENSITY * frac, float(base.t_trans[0]), float(base.t_vib[0]))
    if empty:
        base.counts = np.zeros_like(base.counts)
    return base


def random_state(wl: Workload, seed: int, max_level: int = 3, level_fraction: float = 0.5):
    """Particles in canonical cell order with Maxwellian velocities at each
    cell's T_trans and random low quantum numbers (0..max_level, a fraction
    of modes excited). Every species in the workloads above has at least
    max_level + 1 bound stretch levels for max_level <= 16.
    Returns (cell, species, vel[n,3], levels[n, max_modes])."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5EED]))
    mm = wl.max_modes
    cells, sps = [], []
    for c in range(wl.n_cells):
        for s, k in enumerate(wl.counts[c]):
            cells.append(np.full(int(k), c, np.uint32))
            sps.append(np.full(int(k), s, np.uint8))
    cell = np.concatenate(cells) if cells else np.zeros(0, np.uint32)
    species = np.concatenate(sps) if sps else np.zeros(0, np.uint8)
    n = len(cell)
    mass = np.array([s.mass_kg for s in wl.species])[species]
    sigma = np.sqrt(K_BOLTZ * wl.t_trans[cell] / mass)
    vel = rng.standard_normal((n, 3)) * sigma[:, None]
    levels = np.zeros((n, mm), np.uint16)
    nmodes = np.array([s.n_modes for s in wl.species])[species]
    draw = rng.integers(0, max_level + 1, size=(n, mm))
    on = rng.random((n, mm)) < level_fraction
    mask = np.arange(mm)[None, :] < nmodes[:, None]
    levels[:] = np.where(mask & on, draw, 0)
    return cell, species, vel, levels


def shuffled(cell, species, vel, levels, seed):
    """The same particles in a random order (exercises the counting sort)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x50F7]))
    perm = rng.permutation(len(cell))
    return cell[perm], species[perm], vel[perm], levels[perm]
