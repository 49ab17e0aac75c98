"""Python binding of libhcao.so (ctypes; argument marshalling only).

Every operation runs in the library's HIP kernels on the GPU. The binding
refuses to work without the built library: there is no CPU fallback.
PyTorch is used only to hand the library a HIP stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# HCAO_LIBRARY selects another build of the library (the instrumented
# libhcao_clocks.so of build.py --phase-clocks); default: libhcao.so
LIB_PATH = os.environ.get("HCAO_LIBRARY") or os.path.join(HERE, "libhcao.so")
N_PHASES = 13
PHASES = ("load", "ntc", "temperature", "accept", "sort", "collide", "place", "store", "collide_gather",
          "collide_decide", "collide_relax", "collide_scatter", "collide_write")

ABI_VERSION = 1
MAX_SPECIES = 16
MAX_MODES = 16
MAX_REACTIONS = 32
N_CTR = 8 + MAX_REACTIONS
CTR_CANDIDATES, CTR_COLLISIONS, CTR_TRIALS, CTR_RELAX, CTR_CAPPED, CTR_SUPPRESSED, CTR_BIRTHS, CTR_DEATHS = range(8)
CTR_REACTION0 = 8
FP64, MIXED = 0, 1

STATUS = {0: "HCAO_OK", -1: "HCAO_EINVAL", -2: "HCAO_ESTATE", -3: "HCAO_ENOMEM", -4: "HCAO_EDEVICE",
          -5: "HCAO_ECAPACITY", -6: "HCAO_ELEVEL", -7: "HCAO_ENONFINITE", -8: "HCAO_EUNSUPPORTED",
          -9: "HCAO_EBOUNDS"}

_d, _u32, _u64, _i32 = ctypes.c_double, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
_vp = ctypes.c_void_p
_pd = ctypes.POINTER(ctypes.c_double)


class hcao_config(ctypes.Structure):
    _fields_ = [("abi_version", _u32), ("precision", ctypes.c_int), ("seed", _u64), ("n_cells", _u32),
                ("cell_volume", _pd), ("cell_weight", _pd), ("capacity_per_cell", _u32), ("device", ctypes.c_int),
                ("hip_stream", _vp)]


class hcao_species_desc(ctypes.Structure):
    _fields_ = [("mass_kg", _d), ("dref_m", _d), ("omega", _d), ("Tref_K", _d), ("n_bend", _u32),
                ("bend_theta_K", _pd), ("n_stretch", _u32), ("omega_e_per_m", _pd), ("chi_e", _pd), ("De_J", _pd),
                ("n_levels", ctypes.POINTER(_u32)), ("levels_J", _pd), ("formation_J", _d), ("coupling", _d),
                ("p_vib", _d), ("sampler", ctypes.c_int), ("zeta_rot", _u32), ("p_rot", _d)]


class hcao_reaction_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("reactant", _i32 * 2), ("product", _i32 * 2), ("stretch_mask", _u64),
                ("alpha", _pd), ("steric", _d), ("Ea_J", _d), ("gamma_rot", _d), ("n_samp", _u32),
                ("rec_model", ctypes.c_int)]


class hcao_moments(ctypes.Structure):
    _fields_ = [("n_total", _u64), ("n_species", _u64 * MAX_SPECIES), ("number_density", _d * MAX_SPECIES),
                ("momentum", _d * 3), ("E_trans_J", _d), ("E_kin_J", _d), ("E_vib_J", _d * MAX_SPECIES),
                ("E_formation_J", _d), ("T_trans_K", _d), ("T_vib_K", _d * MAX_SPECIES), ("E_defect_J", _d),
                ("E_rot_J", _d * MAX_SPECIES), ("T_rot_K", _d * MAX_SPECIES)]


class hcao_domain(ctypes.Structure):
    _fields_ = [("nx", _u32), ("ny", _u32), ("nz", _u32), ("periodic", _u32), ("lx", _d), ("ly", _d), ("lz", _d)]


class hcao_inflow(ctypes.Structure):
    _fields_ = [("open_faces", _u32), ("pad", _u32), ("number_density", _vp), ("t_trans_K", _d), ("t_vib_K", _d)]


class hcao_launch_shape(ctypes.Structure):
    _fields_ = [("block", _u32), ("group_slots", _u32), ("steps_per_launch", _u32)]


class HcaoError(RuntimeError):
    def __init__(self, call, code, msg=""):
        super().__init__(f"{call}: {STATUS.get(code, code)} {msg}".strip())
        self.code = code


_lib = None


def load_library():
    """Loads libhcao.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(the HCAO step has no CPU fallback)")
    # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7. If
    # it is loaded first, the library binds to that same runtime (same
    # soname); loading the library first and PyTorch afterwards would start a
    # second runtime that finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    L.hcao_status_string.argtypes = [st]; L.hcao_status_string.restype = ctypes.c_char_p
    L.hcao_last_error.argtypes = [_vp]; L.hcao_last_error.restype = ctypes.c_char_p
    L.hcao_create.argtypes = [ctypes.POINTER(hcao_config), ctypes.POINTER(_vp)]
    L.hcao_add_species.argtypes = [_vp, ctypes.POINTER(hcao_species_desc), ctypes.POINTER(_i32)]
    L.hcao_add_reaction.argtypes = [_vp, ctypes.POINTER(hcao_reaction_desc), ctypes.POINTER(_i32)]
    L.hcao_finalize.argtypes = [_vp]
    L.hcao_load_particles.argtypes = [_vp, _u64, _vp, _vp, _vp, _vp, _vp, _vp]
    L.hcao_set_domain.argtypes = [_vp, ctypes.POINTER(hcao_domain)]
    L.hcao_set_inflow.argtypes = [_vp, ctypes.POINTER(hcao_inflow)]
    L.hcao_read_flux_counts.argtypes = [_vp, _vp]
    L.hcao_read_positions.argtypes = [_vp, _vp]
    L.hcao_read_rotational_energy.argtypes = [_vp, _vp]
    L.hcao_init_thermal.argtypes = [_vp, _vp, _vp, _vp]
    L.hcao_step.argtypes = [_vp, _d, _u32]
    L.hcao_sync.argtypes = [_vp]
    L.hcao_get_counts.argtypes = [_vp, _vp, ctypes.POINTER(_u64)]
    L.hcao_max_modes.argtypes = [_vp]; L.hcao_max_modes.restype = _u32
    L.hcao_step_index.argtypes = [_vp]; L.hcao_step_index.restype = _u32
    L.hcao_read_particles.argtypes = [_vp, _vp, _vp, _vp]
    L.hcao_read_cell_state.argtypes = [_vp, _vp, _vp, _vp]
    L.hcao_read_moments.argtypes = [_vp, _vp, ctypes.POINTER(hcao_moments)]
    L.hcao_read_reaction_counts.argtypes = [_vp, _vp]
    L.hcao_get_levels.argtypes = [_vp, _u32, _u32, _vp, _u32, ctypes.POINTER(_u32)]
    L.hcao_get_pair.argtypes = [_vp, _u32, _u32, _vp]
    L.hcao_get_recombination_table.argtypes = [_vp, _u32, _vp, _u32, ctypes.POINTER(_u32)]
    L.hcao_get_exact_beta.argtypes = [_vp, _u32, _u32, _d, ctypes.POINTER(_d)]
    L.hcao_recombination_exact.argtypes = [_vp, _u32, _d, _d, _u32, _vp, _vp, ctypes.POINTER(_d), ctypes.POINTER(_u64)]
    L.hcao_set_timing.argtypes = [_vp, ctypes.c_int]
    L.hcao_kernel_time.argtypes = [_vp, ctypes.POINTER(_d), ctypes.POINTER(_u64), ctypes.POINTER(_u64)]
    L.hcao_save.argtypes = [_vp, ctypes.c_char_p]
    L.hcao_restore.argtypes = [_vp, ctypes.c_char_p]
    L.hcao_destroy.argtypes = [_vp]; L.hcao_destroy.restype = None
    L.hcao_get_launch_shape.argtypes = [_vp, ctypes.POINTER(hcao_launch_shape)]
    L.hcao_set_launch_shape.argtypes = [_vp, ctypes.POINTER(hcao_launch_shape)]
    L.hcao_autotune.argtypes = [_vp, _d, _u32, ctypes.c_char_p, ctypes.POINTER(hcao_launch_shape)]
    L.hcao_step_graph.argtypes = [_vp, _d, _u32]
    L.hcao_step_static.argtypes = [_vp, _d, _u32]
    L.hcao_read_cell_particles.argtypes = [_vp, _u32, _u32, _vp, _vp, _vp, ctypes.POINTER(_u32)]
    L.hcao_phase_clocks.argtypes = [_vp, _vp, _u32, ctypes.c_int]
    for name in ("hcao_create", "hcao_add_species", "hcao_add_reaction", "hcao_finalize", "hcao_load_particles",
                 "hcao_init_thermal", "hcao_step", "hcao_sync", "hcao_get_counts", "hcao_read_particles",
                 "hcao_read_cell_state", "hcao_read_moments", "hcao_read_reaction_counts", "hcao_get_levels",
                 "hcao_get_pair", "hcao_get_recombination_table", "hcao_set_timing", "hcao_kernel_time", "hcao_save", "hcao_restore",
                 "hcao_get_launch_shape", "hcao_set_launch_shape", "hcao_autotune", "hcao_step_graph",
                 "hcao_read_cell_particles", "hcao_get_exact_beta", "hcao_recombination_exact",
                 "hcao_read_rotational_energy", "hcao_set_domain", "hcao_read_positions", "hcao_set_inflow",
                 "hcao_read_flux_counts", "hcao_phase_clocks", "hcao_step_static"):
        getattr(L, name).restype = st
    _lib = L
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(_vp)


def _dp(a):
    return None if a is None else a.ctypes.data_as(_pd)


def torch_stream():
    """The current PyTorch HIP stream handle (or None)."""
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


class Simulation:
    """One library context: cells, species, reactions and particles on the GPU."""

    def __init__(self, seed: int, n_cells: int, cell_volume, cell_weight, capacity_per_cell: int = 0,
                 device: int = 0, stream=None, precision: int = FP64):
        self._L = load_library()
        self._keep = []
        vol = np.ascontiguousarray(np.broadcast_to(np.asarray(cell_volume, np.float64), (n_cells,)))
        wgt = np.ascontiguousarray(np.broadcast_to(np.asarray(cell_weight, np.float64), (n_cells,)))
        self._keep += [vol, wgt]
        if stream is None:
            stream = torch_stream()
        cfg = hcao_config(ABI_VERSION, precision, int(seed) & (2**64 - 1), n_cells, _dp(vol), _dp(wgt),
                          capacity_per_cell, device, stream)
        h = _vp()
        self._chk("hcao_create", self._L.hcao_create(ctypes.byref(cfg), ctypes.byref(h)), handle=False)
        self._h = h
        self.n_cells = n_cells
        self.n_species = 0
        self.n_reactions = 0
        self.max_modes = 0
        self.precision = precision
        self._n_modes = []

    # -- plumbing --
    def _chk(self, call, rc, handle=True):
        if rc != 0:
            msg = ""
            if handle and getattr(self, "_h", None):
                msg = self._L.hcao_last_error(self._h).decode()
            elif not handle:
                msg = self._L.hcao_last_error(None).decode()
            raise HcaoError(call, rc, msg)

    def close(self):
        if getattr(self, "_h", None):
            self._L.hcao_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up --
    def add_species(self, sp) -> int:
        th = np.asarray(sp.bend_theta_K, np.float64)
        we = np.asarray(sp.omega_e_per_m, np.float64)
        xe = np.asarray(sp.chi_e, np.float64)
        de = np.asarray(sp.De_J, np.float64)
        nl = lv = None
        if getattr(sp, "levels_J", None) is not None:
            nl = np.asarray([len(x) for x in sp.levels_J], np.uint32)
            lv = np.concatenate([np.asarray(x, np.float64) for x in sp.levels_J])
        self._keep += [th, we, xe, de, nl, lv]
        d = hcao_species_desc(sp.mass_kg, sp.dref_m, sp.omega, sp.Tref_K, len(th), _dp(th) if len(th) else None,
                              len(we), _dp(we) if len(we) else None, _dp(xe) if len(xe) else None,
                              _dp(de) if len(de) else None,
                              nl.ctypes.data_as(ctypes.POINTER(_u32)) if nl is not None else None, _dp(lv),
                              sp.formation_J, getattr(sp, "coupling", 0.0), sp.p_vib, sp.sampler,
                              int(getattr(sp, "zeta_rot", 0)), float(getattr(sp, "p_rot", 0.0)))
        i = _i32()
        self._chk("hcao_add_species", self._L.hcao_add_species(self._h, ctypes.byref(d), ctypes.byref(i)))
        self.n_species += 1
        self._n_modes.append(len(th) + len(we))
        return i.value

    def add_reaction(self, rx) -> int:
        al = None if rx.alpha is None else np.asarray(rx.alpha, np.float64)
        self._keep.append(al)
        d = hcao_reaction_desc(rx.kind, (_i32 * 2)(*rx.reactant), (_i32 * 2)(*rx.product), int(rx.stretch_mask),
                               _dp(al), rx.steric, rx.Ea_J, float(getattr(rx, "gamma_rot", 0.0)), getattr(rx, "n_samp", 0),
                               getattr(rx, "rec_model", 0))
        i = _i32()
        self._chk("hcao_add_reaction", self._L.hcao_add_reaction(self._h, ctypes.byref(d), ctypes.byref(i)))
        self.n_reactions += 1
        return i.value

    def finalize(self):
        self._chk("hcao_finalize", self._L.hcao_finalize(self._h))
        self.max_modes = self._L.hcao_max_modes(self._h)

    # -- particles --
    def set_domain(self, nx, ny, nz, lx, ly, lz, periodic=0):
        """Spatial mode (before finalize): box of nx x ny x nz cells."""
        d = hcao_domain(nx, ny, nz, periodic, lx, ly, lz)
        self._chk("hcao_set_domain", self._L.hcao_set_domain(self._h, ctypes.byref(d)))

    def set_inflow(self, open_faces, number_density, t_trans, t_vib):
        """Spatial mode (after finalize): faces 2 axis + side open to a resting
        reservoir of number densities [n_species] m^-3 at t_trans, t_vib."""
        n = np.ascontiguousarray(number_density, np.float64)
        d = hcao_inflow(int(open_faces), 0, n.ctypes.data, float(t_trans), float(t_vib))
        self._chk("hcao_set_inflow", self._L.hcao_set_inflow(self._h, ctypes.byref(d)))

    def flux_counts(self):
        """(admitted, left) through open faces since the last load, init or restore."""
        out = np.zeros(2, np.uint64)
        self._chk("hcao_read_flux_counts", self._L.hcao_read_flux_counts(self._h, _p(out)))
        return int(out[0]), int(out[1])

    def load_particles(self, cell, species, vel, levels, rot=None, pos=None):
        cell = np.ascontiguousarray(cell, np.uint32)
        species = np.ascontiguousarray(species, np.uint8)
        vel = np.ascontiguousarray(vel, np.float64)
        levels = np.ascontiguousarray(levels, np.uint16)
        rot = None if rot is None else np.ascontiguousarray(rot, np.float64)
        pos = None if pos is None else np.ascontiguousarray(pos, np.float64)
        self._chk("hcao_load_particles",
                  self._L.hcao_load_particles(self._h, len(cell), _p(cell), _p(species), _p(vel), _p(levels),
                                              _p(rot), _p(pos)))

    def read_positions(self):
        """Positions [m] of every particle, in read_particles order (spatial mode)."""
        _, tot = self.counts()
        out = np.zeros((tot, 3), np.float64)
        self._chk("hcao_read_positions", self._L.hcao_read_positions(self._h, _p(out)))
        return out

    def read_rotational_energy(self):
        """Rotational energies [J] of every particle, in read_particles order."""
        _, tot = self.counts()
        out = np.zeros(tot, np.float64)
        self._chk("hcao_read_rotational_energy", self._L.hcao_read_rotational_energy(self._h, _p(out)))
        return out

    def init_thermal(self, counts, t_trans, t_vib):
        counts = np.ascontiguousarray(counts, np.uint32)
        tt = np.ascontiguousarray(np.broadcast_to(np.asarray(t_trans, np.float64), (self.n_cells,)))
        tv = np.ascontiguousarray(np.broadcast_to(np.asarray(t_vib, np.float64), (self.n_cells,)))
        self._chk("hcao_init_thermal", self._L.hcao_init_thermal(self._h, _p(counts), _p(tt), _p(tv)))

    def step(self, dt: float, n_steps: int = 1):
        self._chk("hcao_step", self._L.hcao_step(self._h, float(dt), int(n_steps)))

    def step_static(self, dt: float, n_steps: int = 1):
        """The allocation-free step (scratch in the library's fixed device array)."""
        self._chk("hcao_step_static", self._L.hcao_step_static(self._h, float(dt), int(n_steps)))

    def step_graph(self, dt: float, n_steps: int = 1):
        """hcao_step through a captured hipGraph (captured on first use per (dt, n_steps))."""
        self._chk("hcao_step_graph", self._L.hcao_step_graph(self._h, float(dt), int(n_steps)))

    def launch_shape(self):
        sh = hcao_launch_shape()
        self._chk("hcao_get_launch_shape", self._L.hcao_get_launch_shape(self._h, ctypes.byref(sh)))
        return {"block": sh.block, "group_slots": sh.group_slots, "steps_per_launch": sh.steps_per_launch}

    def set_launch_shape(self, block: int = 64, group_slots: int = 1024, steps_per_launch: int = 0):
        sh = hcao_launch_shape(block, group_slots, steps_per_launch)
        self._chk("hcao_set_launch_shape", self._L.hcao_set_launch_shape(self._h, ctypes.byref(sh)))

    def autotune(self, dt: float, trial_steps: int = 5, cache_path=None):
        sh = hcao_launch_shape()
        cp = None if cache_path is None else str(cache_path).encode()
        self._chk("hcao_autotune", self._L.hcao_autotune(self._h, float(dt), int(trial_steps), cp, ctypes.byref(sh)))
        return {"block": sh.block, "group_slots": sh.group_slots, "steps_per_launch": sh.steps_per_launch}

    def sync(self):
        self._chk("hcao_sync", self._L.hcao_sync(self._h))

    @property
    def step_index(self) -> int:
        return self._L.hcao_step_index(self._h)

    def counts(self):
        per = np.zeros(self.n_cells, np.uint64)
        tot = _u64()
        self._chk("hcao_get_counts", self._L.hcao_get_counts(self._h, _p(per), ctypes.byref(tot)))
        return per, tot.value

    def read_particles(self):
        """Returns (counts per cell, species, vel[n,3], levels[n, max_modes]) in canonical order."""
        per, tot = self.counts()
        sp = np.zeros(tot, np.uint8)
        v = np.zeros((tot, 3), np.float64)
        lv = np.zeros((tot, max(self.max_modes, 1)), np.uint16)
        self._chk("hcao_read_particles", self._L.hcao_read_particles(self._h, _p(sp), _p(v), _p(lv)))
        return per.astype(np.int64), sp, v, lv[:, :self.max_modes]

    def read_cell(self, cell: int, max_n: int = 1 << 20):
        """(species, vel[n,3], levels[n, max_modes]) of one cell in canonical order."""
        mm = max(self.max_modes, 1)
        sp = np.zeros(max_n, np.uint8)
        v = np.zeros((max_n, 3), np.float64)
        lv = np.zeros((max_n, mm), np.uint16)
        n = _u32()
        self._chk("hcao_read_cell_particles", self._L.hcao_read_cell_particles(
            self._h, int(cell), int(max_n), _p(sp), _p(v), _p(lv), ctypes.byref(n)))
        k = min(n.value, max_n)
        return sp[:k], v[:k], lv[:k, :self.max_modes]

    def cell_state(self):
        sg = np.zeros(self.n_cells, np.float64)
        rem = np.zeros(self.n_cells, np.float64)
        ctr = np.zeros((self.n_cells, N_CTR), np.uint64)
        self._chk("hcao_read_cell_state", self._L.hcao_read_cell_state(self._h, _p(sg), _p(rem), _p(ctr)))
        return sg, rem, ctr

    def moments(self, per_cell: bool = False):
        tot = hcao_moments()
        arr = (hcao_moments * self.n_cells)() if per_cell else None
        self._chk("hcao_read_moments", self._L.hcao_read_moments(
            self._h, ctypes.cast(arr, _vp) if per_cell else None, ctypes.byref(tot)))
        return (tot, list(arr)) if per_cell else tot

    def moments_per_cell(self):
        """Per-cell moments as a numpy structured array (fields of hcao_moments)."""
        tot = hcao_moments()
        arr = (hcao_moments * self.n_cells)()
        self._chk("hcao_read_moments", self._L.hcao_read_moments(self._h, ctypes.cast(arr, _vp), ctypes.byref(tot)))
        return np.ctypeslib.as_array(arr).copy()

    def zero_point(self, species) -> float:
        """Zero-point energy of a species [J]: the sum of its modes' ground levels."""
        return float(sum(self.levels(species, m, 1)[0] for m in range(self._n_modes[species])))

    def total_energy(self, m=None, with_defect: bool = True) -> float:
        """Kinetic + vibrational (zero point included) + rotational + formation
        energy of all particles [J], plus, by default, the energy the mixed
        form still owes them."""
        m = self.moments() if m is None else m
        e = m.E_kin_J + m.E_formation_J
        for s in range(self.n_species):
            e += m.E_vib_J[s] + m.n_species[s] * self.zero_point(s) + m.E_rot_J[s]
        return e + (m.E_defect_J if with_defect else 0.0)

    def reaction_counts(self):
        out = np.zeros(max(self.n_reactions, 1), np.uint64)
        self._chk("hcao_read_reaction_counts", self._L.hcao_read_reaction_counts(self._h, _p(out)))
        return out[:self.n_reactions]

    def levels(self, species, mode, max_n=1024):
        out = np.zeros(max_n, np.float64)
        n = _u32()
        self._chk("hcao_get_levels", self._L.hcao_get_levels(self._h, species, mode, _p(out), max_n,
                                                              ctypes.byref(n)))
        return out[:min(n.value, max_n)]

    def pair(self, a, b):
        out = np.zeros(8, np.float64)
        self._chk("hcao_get_pair", self._L.hcao_get_pair(self._h, a, b, _p(out)))
        return dict(zip(("mr", "hm", "msum", "wa", "wb", "csg", "esg", "q"), out))

    def exact_beta(self, species, partner, e_J):
        """Inverse temperature of the EXACT sampler's proposal (host table)."""
        b = _d()
        self._chk("hcao_get_exact_beta", self._L.hcao_get_exact_beta(self._h, species, partner, float(e_J),
                                                                      ctypes.byref(b)))
        return b.value

    def recombination_exact(self, species, de_J, omega, temps):
        """Eq. recomb-correct on the device: (probabilities, device ms, records)."""
        t = np.ascontiguousarray(temps, np.float64)
        p = np.zeros_like(t)
        ms, nrec = _d(), _u64()
        self._chk("hcao_recombination_exact", self._L.hcao_recombination_exact(
            self._h, species, float(de_J), float(omega), len(t), _p(t), _p(p), ctypes.byref(ms), ctypes.byref(nrec)))
        return p, ms.value, nrec.value

    def recombination_table(self, reaction):
        out = np.zeros(self.n_species * 1024, np.float64)
        n = _u32()
        self._chk("hcao_get_recombination_table", self._L.hcao_get_recombination_table(
            self._h, reaction, _p(out), len(out), ctypes.byref(n)))
        return out[:n.value].reshape(self.n_species, -1)

    def set_timing(self, enable: bool):
        self._chk("hcao_set_timing", self._L.hcao_set_timing(self._h, int(enable)))

    def kernel_time(self):
        """(elapsed ms, launches, steps) of the step kernel since set_timing(True)."""
        ms = _d()
        n = _u64()
        k = _u64()
        self._chk("hcao_kernel_time", self._L.hcao_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n),
                                                                ctypes.byref(k)))
        return ms.value, n.value, k.value

    def phase_clocks(self, reset: bool = False):
        """Per-phase clock sums of the step kernel (instrumented builds only;
        raises HcaoError HCAO_EUNSUPPORTED otherwise)."""
        out = np.zeros(N_PHASES, np.uint64)
        self._chk("hcao_phase_clocks", self._L.hcao_phase_clocks(self._h, _p(out), N_PHASES, int(reset)))
        return dict(zip(PHASES, (int(x) for x in out)))

    def save(self, path):
        self._chk("hcao_save", self._L.hcao_save(self._h, str(path).encode()))

    def restore(self, path):
        self._chk("hcao_restore", self._L.hcao_restore(self._h, str(path).encode()))


def from_workload(wl, seed: Optional[int] = None, capacity_per_cell: Optional[int] = None, stream=None,
                  precision: int = FP64):
    """Builds a Simulation with the species and reactions of a workloads.Workload."""
    cap = wl.capacity_per_cell if capacity_per_cell is None else capacity_per_cell
    s = Simulation(wl.seed if seed is None else seed, wl.n_cells, wl.cell_volume, wl.cell_weight, cap,
                   stream=stream, precision=precision)
    if getattr(wl, "domain", None) is not None:
        s.set_domain(*wl.domain)
    for sp in wl.species:
        s.add_species(sp)
    for rx in wl.reactions:
        s.add_reaction(rx)
    s.finalize()
    if getattr(wl, "inflow", None) is not None:
        s.set_inflow(*wl.inflow)
    return s
