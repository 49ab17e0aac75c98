"""fp64 CPU oracle of the HCAO DSMC collision step (ctypes wrapper).

TEST INFRASTRUCTURE: only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg use this package. The GPU library never imports
it and shares no code with it. The arithmetic lives in ``hcao_oracle.c``;
this module only marshals arguments.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hcao_oracle.c")
# ORACLE_LIBRARY names a separately compiled build of hcao_oracle.c (the
# mutation tests load copies with planted mistakes); build() leaves it alone
_ALT = os.environ.get("ORACLE_LIBRARY")
_LIB = _ALT or os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-Wall", "-Wextra", "-Wno-unused-parameter"]

SAMPLER_AUTO, SAMPLER_JOINT, SAMPLER_GIBBS, SAMPLER_EXACT = 0, 1, 2, 3
RX_DISSOCIATION, RX_EXCHANGE, RX_RECOMBINATION = 0, 1, 2
CTR_CANDIDATES, CTR_COLLISIONS, CTR_TRIALS, CTR_RELAX, CTR_CAPPED, CTR_SUPPRESSED, CTR_BIRTHS, CTR_DEATHS = range(8)
CTR_REACTION0 = 8
MAX_REACTIONS = 32
N_CTR = 8 + MAX_REACTIONS


def compile_to(src: str, out: str) -> str:
    """Compile an oracle source file with gcc (IEEE fp64: no contraction, no
    fast-math) into the shared library out."""
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle (unless ORACLE_LIBRARY names another build)."""
    if _ALT:
        return _LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_to(_SRC, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, u32, u64, i32 = ctypes.c_double, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
        vp = ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [u32, u32, vp, vp]
        L.orc_detlog.argtypes = [d]; L.orc_detlog.restype = d
        L.orc_detexp.argtypes = [d]; L.orc_detexp.restype = d
        L.orc_detpow.argtypes = [d, d]; L.orc_detpow.restype = d
        L.orc_feistel_index.argtypes = [u32, vp, u32]; L.orc_feistel_index.restype = u32
        L.orc_gibbs_propose.argtypes = [u32, ctypes.c_double, ctypes.c_double]; L.orc_gibbs_propose.restype = u32
        L.orc_exact_beta.argtypes = [vp, u32, d, d]; L.orc_exact_beta.restype = d
        L.orc_create.argtypes = [u64, u32, vp, vp, u32, P(vp)]
        L.orc_destroy.argtypes = [vp]; L.orc_destroy.restype = None
        L.orc_add_species.argtypes = [vp, d, d, d, d, u32, vp, u32, vp, vp, vp, vp, vp, d, d, ctypes.c_int]
        L.orc_add_reaction.argtypes = [vp, ctypes.c_int, vp, vp, u64, vp, d, d, u32]
        L.orc_finalize.argtypes = [vp]
        L.orc_load.argtypes = [vp, u64, vp, vp, vp, vp, vp, vp]
        L.orc_set_domain.argtypes = [vp, u32, u32, u32, d, d, d, u32]; L.orc_set_domain.restype = ctypes.c_int
        L.orc_read_pos.argtypes = [vp, u32, vp]; L.orc_read_pos.restype = ctypes.c_int
        L.orc_set_inflow.argtypes = [vp, u32, vp, d, d]; L.orc_set_inflow.restype = ctypes.c_int
        L.orc_flux_counts.argtypes = [vp, vp]; L.orc_flux_counts.restype = ctypes.c_int
        L.orc_set_rotation.argtypes = [vp, u32, u32, d]; L.orc_set_rotation.restype = ctypes.c_int
        L.orc_set_gamma_rot.argtypes = [vp, u32, d]; L.orc_set_gamma_rot.restype = ctypes.c_int
        L.orc_read_rot.argtypes = [vp, u32, vp]; L.orc_read_rot.restype = ctypes.c_int
        L.orc_rot_energy.argtypes = [vp, u32, vp]; L.orc_rot_energy.restype = ctypes.c_int
        L.orc_collide_rot_batch.argtypes = [vp, u32] + [vp] * 13; L.orc_collide_rot_batch.restype = ctypes.c_int
        L.orc_init_thermal.argtypes = [vp, vp, vp, vp]
        L.orc_step.argtypes = [vp, d, u32]
        L.orc_set_threads.argtypes = [vp, ctypes.c_int]; L.orc_set_threads.restype = ctypes.c_int
        L.orc_max_modes.argtypes = [vp]; L.orc_max_modes.restype = u32
        L.orc_count.argtypes = [vp, u32]; L.orc_count.restype = u64
        L.orc_step_index.argtypes = [vp]; L.orc_step_index.restype = u32
        L.orc_read_cell.argtypes = [vp, u32, vp, vp, vp]
        L.orc_read_cell_state.argtypes = [vp, u32, vp, vp, vp]
        L.orc_levels.argtypes = [vp, u32, u32, vp, u32]
        L.orc_species_info.argtypes = [vp, u32, vp, vp, vp]
        L.orc_pair_info.argtypes = [vp, u32, u32, vp]
        L.orc_moments.argtypes = [vp, u32, vp]
        L.orc_tvib.argtypes = [vp, u32, d, vp]
        L.orc_relax_batch.argtypes = [vp, u32, d, ctypes.c_int, u32, vp, vp, vp, vp, vp]
        L.orc_relax_chain.argtypes = [vp, u32, d, ctypes.c_int, u32, u32, vp, vp, vp, u32]
        L.orc_collide_batch.argtypes = [vp, u32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_collide3_batch.argtypes = [vp, u32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, d, d]
        L.orc_collide3_batch.restype = ctypes.c_int
        L.orc_gamma_q.argtypes = [d, d]; L.orc_gamma_q.restype = d
        L.orc_wr_rho.argtypes = [vp, u32, d]; L.orc_wr_rho.restype = d
        L.orc_wr_probability.argtypes = [vp, u32, d, d, u32, d]; L.orc_wr_probability.restype = d
        L.orc_q_vib.argtypes = [vp, u32, d]; L.orc_q_vib.restype = d
        L.orc_rec_exact_probability.argtypes = [vp, u32, d, d, d]; L.orc_rec_exact_probability.restype = d
        L.orc_rec_factor.argtypes = [vp, u32, u32, d]; L.orc_rec_factor.restype = d
        L.orc_rec_table.argtypes = [vp, u32, vp]; L.orc_rec_table.restype = ctypes.c_int
        L.orc_equilibrium_constant.argtypes = [vp, u32, d]; L.orc_equilibrium_constant.restype = d
        L.orc_forward_rate.argtypes = [vp, u32, u32, d]; L.orc_forward_rate.restype = d
        L.orc_forward_probability.argtypes = [vp, u32, u32, d]; L.orc_forward_probability.restype = d
        L.orc_rec_node_temperature.argtypes = [vp, u32]; L.orc_rec_node_temperature.restype = d
        L.orc_cell_temperature.argtypes = [vp, u32]; L.orc_cell_temperature.restype = d
        L.orc_cell_sums.argtypes = [vp, u32, ctypes.c_int, vp]; L.orc_cell_sums.restype = ctypes.c_int
        L.orc_draw_unit_vectors.argtypes = [u64, u32, vp]; L.orc_draw_unit_vectors.restype = None
        L.orc_draw_three_body_shares.argtypes = [u64, u32, vp]; L.orc_draw_three_body_shares.restype = None
        for name in ("orc_create", "orc_add_species", "orc_add_reaction", "orc_finalize", "orc_load",
                     "orc_init_thermal", "orc_step", "orc_read_cell", "orc_read_cell_state", "orc_levels",
                     "orc_species_info", "orc_pair_info", "orc_moments", "orc_tvib", "orc_relax_batch",
                     "orc_relax_chain", "orc_collide_batch"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, call, code):
        super().__init__(f"{call} failed with code {code}")
        self.code = code


def _chk(call, rc):
    if rc < 0:
        raise OracleError(call, rc)
    return rc


# ---- primitives -----------------------------------------------------------

def philox(key, ctr):
    out = np.zeros(4, np.uint32)
    c = np.asarray(ctr, np.uint32)
    lib().orc_philox4x32_10(int(key[0]), int(key[1]), _p(c), _p(out))
    return out


def detlog(x):
    return lib().orc_detlog(float(x))


def detexp(x):
    return lib().orc_detexp(float(x))


def detpow(x, y):
    return lib().orc_detpow(float(x), float(y))


def gamma_q(a, x):
    return lib().orc_gamma_q(float(a), float(x))


def gibbs_propose(top, c, u):
    return lib().orc_gibbs_propose(int(top), float(c), float(u))


def draw_unit_vectors(seed, n):
    out = np.zeros((n, 3), np.float64)
    lib().orc_draw_unit_vectors(int(seed), int(n), _p(out))
    return out


def draw_three_body_shares(seed, n):
    out = np.zeros(n, np.float64)
    lib().orc_draw_three_body_shares(int(seed), int(n), _p(out))
    return out


def feistel_index(n, keys, i):
    k = np.asarray(keys, np.uint32)
    return lib().orc_feistel_index(int(n), _p(k), int(i))


# ---- context ----------------------------------------------------------------

@dataclass
class Moments:
    momentum: np.ndarray
    sum_mv2: float
    mass: float
    formation: float
    count: np.ndarray
    evib: np.ndarray
    evib_above_zpe: np.ndarray


class Oracle:
    """One oracle simulation: species, reactions, cells and particles."""

    def __init__(self, seed, n_cells, volume, weight, capacity_per_cell=0):
        vol = np.broadcast_to(np.asarray(volume, np.float64), (n_cells,)).copy()
        wgt = np.broadcast_to(np.asarray(weight, np.float64), (n_cells,)).copy()
        h = ctypes.c_void_p()
        _chk("orc_create", lib().orc_create(int(seed), int(n_cells), _p(vol), _p(wgt), int(capacity_per_cell),
                                            ctypes.byref(h)))
        self._h = h
        self.n_cells = n_cells
        self.n_species = 0
        self.n_reactions = 0

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_species(self, sp):
        """sp: a workloads.Species-like object."""
        th = np.asarray(sp.bend_theta_K, np.float64)
        we = np.asarray(sp.omega_e_per_m, np.float64)
        xe = np.asarray(sp.chi_e, np.float64)
        de = np.asarray(sp.De_J, np.float64)
        nl = None
        lv = None
        if getattr(sp, "levels_J", None) is not None:
            nl = np.asarray([len(x) for x in sp.levels_J], np.uint32)
            lv = np.concatenate([np.asarray(x, np.float64) for x in sp.levels_J])
        _chk("orc_add_species", lib().orc_add_species(
            self._h, sp.mass_kg, sp.dref_m, sp.omega, sp.Tref_K, len(th), _p(th) if len(th) else None,
            len(we), _p(we) if len(we) else None, _p(xe) if len(xe) else None, _p(de) if len(de) else None,
            _p(nl), _p(lv), sp.formation_J, sp.p_vib, sp.sampler))
        if getattr(sp, "zeta_rot", 0):
            _chk("orc_set_rotation", lib().orc_set_rotation(self._h, self.n_species, int(sp.zeta_rot), float(sp.p_rot)))
        self.n_species += 1
        return self.n_species - 1

    def add_reaction(self, rx):
        r = np.asarray(rx.reactant, np.int32)
        p = np.asarray(rx.product, np.int32)
        al = None if rx.alpha is None else np.asarray(rx.alpha, np.float64)
        _chk("orc_add_reaction", lib().orc_add_reaction(self._h, rx.kind, _p(r), _p(p), int(rx.stretch_mask),
                                                        _p(al), rx.steric, rx.Ea_J, int(getattr(rx, "n_samp", 0))))
        if getattr(rx, "gamma_rot", 0.0):
            _chk("orc_set_gamma_rot", lib().orc_set_gamma_rot(self._h, self.n_reactions, float(rx.gamma_rot)))
        self.n_reactions += 1
        return self.n_reactions - 1

    def finalize(self):
        _chk("orc_finalize", lib().orc_finalize(self._h))
        self.max_modes = lib().orc_max_modes(self._h)

    def set_domain(self, nx, ny, nz, lx, ly, lz, periodic=0):
        _chk("orc_set_domain", lib().orc_set_domain(self._h, nx, ny, nz, float(lx), float(ly), float(lz),
                                                    int(periodic)))

    def set_inflow(self, open_faces, number_density, t_trans, t_vib):
        n = np.ascontiguousarray(number_density, np.float64)
        _chk("orc_set_inflow", lib().orc_set_inflow(self._h, int(open_faces), _p(n), float(t_trans), float(t_vib)))

    def flux_counts(self):
        out = np.zeros(2, np.uint64)
        _chk("orc_flux_counts", lib().orc_flux_counts(self._h, _p(out)))
        return int(out[0]), int(out[1])

    def load(self, cell, species, vel, levels, rot=None, pos=None):
        cell = np.ascontiguousarray(cell, np.uint32)
        species = np.ascontiguousarray(species, np.uint8)
        vel = np.ascontiguousarray(vel, np.float64)
        levels = np.ascontiguousarray(levels, np.uint16)
        rot = None if rot is None else np.ascontiguousarray(rot, np.float64)
        pos = None if pos is None else np.ascontiguousarray(pos, np.float64)
        _chk("orc_load", lib().orc_load(self._h, len(cell), _p(cell), _p(species), _p(vel), _p(levels), _p(rot),
                                        _p(pos)))

    def read_pos(self, cell):
        out = np.zeros((self.count(cell), 3), np.float64)
        _chk("orc_read_pos", lib().orc_read_pos(self._h, cell, _p(out)))
        return out

    def read_rot(self, cell):
        out = np.zeros(self.count(cell), np.float64)
        _chk("orc_read_rot", lib().orc_read_rot(self._h, cell, _p(out)))
        return out

    def rot_energy(self, cell):
        out = np.zeros(self.n_species, np.float64)
        _chk("orc_rot_energy", lib().orc_rot_energy(self._h, cell, _p(out)))
        return out

    def init_thermal(self, counts, t_trans, t_vib):
        counts = np.ascontiguousarray(counts, np.uint32)
        tt = np.ascontiguousarray(np.broadcast_to(np.asarray(t_trans, np.float64), (self.n_cells,)))
        tv = np.ascontiguousarray(np.broadcast_to(np.asarray(t_vib, np.float64), (self.n_cells,)))
        _chk("orc_init_thermal", lib().orc_init_thermal(self._h, _p(counts), _p(tt), _p(tv)))

    def step(self, dt, n_steps=1):
        _chk("orc_step", lib().orc_step(self._h, float(dt), int(n_steps)))

    def set_threads(self, n):
        """OpenMP threads over cells in step() (cells are independent, so the
        result does not depend on n)."""
        _chk("orc_set_threads", lib().orc_set_threads(self._h, int(n)))

    @property
    def step_index(self):
        return lib().orc_step_index(self._h)

    def count(self, cell):
        return lib().orc_count(self._h, cell)

    def read_cell(self, cell):
        n = self.count(cell)
        sp = np.zeros(n, np.uint8)
        v = np.zeros((n, 3), np.float64)
        lv = np.zeros((n, self.max_modes), np.uint16)
        _chk("orc_read_cell", lib().orc_read_cell(self._h, cell, _p(sp), _p(v), _p(lv)))
        return sp, v, lv

    def read_all(self):
        parts = [self.read_cell(c) for c in range(self.n_cells)]
        counts = np.array([len(p[0]) for p in parts], np.int64)
        return (counts, np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]),
                np.concatenate([p[2] for p in parts]))

    def cell_state(self, cell):
        sg = ctypes.c_double()
        rem = ctypes.c_double()
        ctr = np.zeros(N_CTR, np.uint64)
        _chk("orc_read_cell_state", lib().orc_read_cell_state(self._h, cell, ctypes.byref(sg), ctypes.byref(rem),
                                                              _p(ctr)))
        return sg.value, rem.value, ctr

    def counters(self):
        return np.stack([self.cell_state(c)[2] for c in range(self.n_cells)])

    def levels(self, species, mode, max_n=1024):
        out = np.zeros(max_n, np.float64)
        n = _chk("orc_levels", lib().orc_levels(self._h, species, mode, _p(out), max_n))
        return out[:n]

    def species_info(self, species):
        z = ctypes.c_double()
        nm = ctypes.c_uint32()
        smp = ctypes.c_uint32()
        _chk("orc_species_info", lib().orc_species_info(self._h, species, ctypes.byref(z), ctypes.byref(nm),
                                                        ctypes.byref(smp)))
        return z.value, nm.value, smp.value

    def pair_info(self, a, b):
        out = np.zeros(8, np.float64)
        _chk("orc_pair_info", lib().orc_pair_info(self._h, a, b, _p(out)))
        return dict(zip(("mr", "hm", "msum", "wa", "wb", "csg", "esg", "q"), out))

    def moments(self, cell):
        out = np.zeros(6 + 3 * self.n_species, np.float64)
        _chk("orc_moments", lib().orc_moments(self._h, cell, _p(out)))
        per = out[6:].reshape(self.n_species, 3)
        return Moments(out[0:3].copy(), out[3], out[4], out[5], per[:, 0].copy(), per[:, 1].copy(),
                       per[:, 2].copy())

    def tvib(self, species, mean_evib_above_ground):
        t = ctypes.c_double()
        _chk("orc_tvib", lib().orc_tvib(self._h, species, float(mean_evib_above_ground), ctypes.byref(t)))
        return t.value

    def exact_beta(self, species, q, ep):
        return lib().orc_exact_beta(self._h, int(species), float(q), float(ep))

    def relax_batch(self, species, q, sampler, e_tr, lvl_in):
        e_tr = np.ascontiguousarray(e_tr, np.float64)
        n = len(e_tr)
        lvl_in = np.ascontiguousarray(lvl_in, np.uint16)
        lvl_out = np.zeros_like(lvl_in)
        e_out = np.zeros(n, np.float64)
        trials = np.zeros(n, np.uint64)
        _chk("orc_relax_batch", lib().orc_relax_batch(self._h, species, float(q), int(sampler), n, _p(e_tr),
                                                      _p(lvl_in), _p(lvl_out), _p(e_out), _p(trials)))
        return lvl_out, e_out, trials

    def relax_chain(self, species, q, sampler, e_tr, lvl0, chain=0, hist_stride=0):
        """Runs one heat-bath chain; returns (histogram or None, final levels)."""
        e_tr = np.ascontiguousarray(e_tr, np.float64)
        state = np.ascontiguousarray(lvl0, np.uint16).copy()
        nm = len(state)
        hist = np.zeros((nm, hist_stride), np.uint64) if hist_stride else None
        _chk("orc_relax_chain", lib().orc_relax_chain(self._h, species, float(q), int(sampler), int(chain),
                                                      len(e_tr), _p(e_tr), _p(state), _p(hist), hist_stride))
        return hist, state

    def wr_rho(self, species, e):
        return lib().orc_wr_rho(self._h, species, float(e))

    def wr_probability(self, species, de, omega, n_samp, t):
        return lib().orc_wr_probability(self._h, species, float(de), float(omega), int(n_samp), float(t))

    def rec_exact_probability(self, species, de, omega, t):
        return lib().orc_rec_exact_probability(self._h, species, float(de), float(omega), float(t))

    def q_vib(self, species, t):
        return lib().orc_q_vib(self._h, species, float(t))

    def rec_factor(self, reaction, third, t):
        return lib().orc_rec_factor(self._h, reaction, third, float(t))

    def equilibrium_constant(self, reaction, t):
        return lib().orc_equilibrium_constant(self._h, int(reaction), float(t))

    def forward_rate(self, reaction, third, t):
        return lib().orc_forward_rate(self._h, int(reaction), int(third), float(t))

    def forward_probability(self, reaction, third, t):
        return lib().orc_forward_probability(self._h, int(reaction), int(third), float(t))

    def rec_node_temperature(self, i):
        return lib().orc_rec_node_temperature(self._h, int(i))

    def cell_temperature(self, cell):
        return lib().orc_cell_temperature(self._h, int(cell))

    def cell_sums(self, cell, direct=False):
        out = np.zeros(5, np.float64)
        _chk("orc_cell_sums", lib().orc_cell_sums(self._h, int(cell), int(direct), _p(out)))
        return out

    def rec_table(self, reaction):
        out = np.zeros(self.n_species * 1024, np.float64)
        _chk("orc_rec_table", lib().orc_rec_table(self._h, reaction, _p(out)))
        return out.reshape(self.n_species, 1024)

    def collide3_batch(self, sp, vel, lvl, m_sp, m_vel, t_cell, n_cell):
        """collide_batch with a third body per item (recombination)."""
        sp = np.ascontiguousarray(sp, np.uint8)
        n = len(sp) // 2
        vel = np.ascontiguousarray(vel, np.float64)
        lvl = np.ascontiguousarray(lvl, np.uint16)
        m_sp = np.ascontiguousarray(m_sp, np.uint8)
        m_vel = np.ascontiguousarray(m_vel, np.float64).copy()
        sp_o = np.zeros_like(sp)
        vel_o = np.zeros_like(vel)
        lvl_o = np.zeros_like(lvl)
        rx = np.zeros(n, np.int32)
        bsp = np.zeros(n, np.uint8)
        bvel = np.zeros((n, 3), np.float64)
        blvl = np.zeros((n, self.max_modes), np.uint16)
        _chk("orc_collide3_batch", lib().orc_collide3_batch(
            self._h, n, _p(sp), _p(vel), _p(lvl), _p(sp_o), _p(vel_o), _p(lvl_o), _p(rx), _p(bsp), _p(bvel),
            _p(blvl), _p(m_sp), _p(m_vel), float(t_cell), float(n_cell)))
        return sp_o, vel_o, lvl_o, rx, m_vel

    def collide_batch(self, sp, vel, lvl):
        sp = np.ascontiguousarray(sp, np.uint8)
        n = len(sp) // 2
        vel = np.ascontiguousarray(vel, np.float64)
        lvl = np.ascontiguousarray(lvl, np.uint16)
        sp_o = np.zeros_like(sp)
        vel_o = np.zeros_like(vel)
        lvl_o = np.zeros_like(lvl)
        rx = np.zeros(n, np.int32)
        bsp = np.zeros(n, np.uint8)
        bvel = np.zeros((n, 3), np.float64)
        blvl = np.zeros((n, self.max_modes), np.uint16)
        _chk("orc_collide_batch", lib().orc_collide_batch(self._h, n, _p(sp), _p(vel), _p(lvl), _p(sp_o), _p(vel_o),
                                                          _p(lvl_o), _p(rx), _p(bsp), _p(bvel), _p(blvl)))
        return sp_o, vel_o, lvl_o, rx, bsp, bvel, blvl

    def collide_rot_batch(self, sp, vel, lvl, rot):
        """collide_batch with rotational energies: returns also rot out and the
        newborns' rotational energies."""
        sp = np.ascontiguousarray(sp, np.uint8)
        n = len(sp) // 2
        vel = np.ascontiguousarray(vel, np.float64)
        lvl = np.ascontiguousarray(lvl, np.uint16)
        rot = np.ascontiguousarray(rot, np.float64)
        sp_o, vel_o, lvl_o, rot_o = np.zeros_like(sp), np.zeros_like(vel), np.zeros_like(lvl), np.zeros_like(rot)
        rx = np.zeros(n, np.int32)
        bsp = np.zeros(n, np.uint8)
        bvel = np.zeros((n, 3), np.float64)
        blvl = np.zeros((n, self.max_modes), np.uint16)
        brot = np.zeros(n, np.float64)
        _chk("orc_collide_rot_batch", lib().orc_collide_rot_batch(
            self._h, n, _p(sp), _p(vel), _p(lvl), _p(rot), _p(sp_o), _p(vel_o), _p(lvl_o), _p(rot_o), _p(rx),
            _p(bsp), _p(bvel), _p(blvl), _p(brot)))
        return sp_o, vel_o, lvl_o, rot_o, rx, bsp, bvel, blvl, brot


def from_workload(wl, seed=None, capacity_per_cell=None):
    """Builds an Oracle with the species and reactions of a workloads.Workload."""
    cap = getattr(wl, "capacity_per_cell", 0) if capacity_per_cell is None else capacity_per_cell
    o = Oracle(wl.seed if seed is None else seed, wl.n_cells, wl.cell_volume, wl.cell_weight, cap)
    if getattr(wl, "domain", None) is not None:
        o.set_domain(*wl.domain)
    for sp in wl.species:
        o.add_species(sp)
    for rx in wl.reactions:
        o.add_reaction(rx)
    o.finalize()
    if getattr(wl, "inflow", None) is not None:
        o.set_inflow(*wl.inflow)
    return o
