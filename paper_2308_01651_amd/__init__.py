"""MI355X-native monodomain time step (lifex-ep method) behind a C ABI.

Python binding with the same names as include/ep.h; argument marshalling
only.  Every step of the time-stepping path runs in the HIP kernels of
libep_mi355x.so; there is no CPU fallback: if the library is missing, import
fails.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import EpError, EpStats, check, lib

# constants (include/ep.h)
EP_TET4, EP_TET10, EP_HEX8, EP_HEX27, EP_HEX64, EP_HEX125, EP_HEX216, EP_HEX343 = 4, 10, 8, 27, 64, 125, 216, 343
EP_PASSIVE, EP_AP, EP_BO, EP_TTP06 = 0, 1, 2, 3
EP_CELL_EPI, EP_CELL_ENDO, EP_CELL_MID = 0, 1, 2
EP_CUBE, EP_SPHERE, EP_GAUSS = 0, 1, 2
EP_FP64, EP_MIXED = 0, 1
EP_JACOBI = 0
EP_BJACOBI = 1
EP_DTYPE_F64, EP_DTYPE_F32 = 0, 1
EP_FMT_AUTO, EP_FMT_SELL, EP_FMT_DIA, EP_FMT_MF = 0, 1, 2, 3
EP_OPT_MATRIX_FORMAT, EP_OPT_INNER_RTOL, EP_OPT_MAX_OUTER, EP_OPT_PHASE_TIMERS = 1, 2, 3, 4
EP_OPT_KERNEL_TIMERS = 5
EP_OPT_IONIC_NPT, EP_OPT_TILE_MAP, EP_OPT_GRAPH, EP_OPT_IONIC_SCHEME, EP_OPT_IONIC_FP64 = 6, 7, 8, 9, 10
EP_OPT_CG_VARIANT, EP_OPT_INITIAL_GUESS = 11, 12
EP_X0_EXT, EP_X0_EXTRAP3 = 0, 1
EP_CG_AUTO, EP_CG_PIPELINED, EP_CG_CHRONOPOULOS_GEAR = 0, 1, 2
EP_IONIC_RUSH_LARSEN, EP_IONIC_BDF = 0, 1
EP_MAX_REGIONS = 8
KERNEL_KINDS = ["ionic", "rhs", "cg_spmv", "cg_update", "activation", "ir_residual", "cg_finalize", "cg_pipe"]

MODEL_IDS = {"passive": EP_PASSIVE, "ap": EP_AP, "bo": EP_BO, "ttp06": EP_TTP06}
CELL_IDS = {"": EP_CELL_EPI, "epi": EP_CELL_EPI, "endo": EP_CELL_ENDO, "mid": EP_CELL_MID}


def _pd(a):
    return a.ctypes.data_as(_lib.PD)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Simulation:
    """One monodomain simulation on one GPU (wraps ep_sim)."""

    def __init__(self, device: int = 0, stream=None):
        h = C.c_void_p()
        check(lib.ep_sim_create(int(device), C.c_void_p(stream) if stream else None, C.byref(h)),
              "ep_sim_create")
        self._h = h
        self.n_nodes = 0
        self.bdf = 1

    # -- configuration ---------------------------------------------------------
    def upload_mesh(self, elem: int, xyz, conn, material=None):
        """material: optional per-element subdomain labels 0..EP_MAX_REGIONS-1."""
        xyz = _f64(xyz)
        conn = np.ascontiguousarray(conn, dtype=np.int32)
        self.n_nodes = xyz.shape[0]
        mat = None if material is None else np.ascontiguousarray(material, dtype=np.int32)
        check(lib.ep_sim_upload_mesh(self._h, int(elem), xyz.shape[0], _pd(xyz), conn.shape[0],
                                     conn.ctypes.data_as(_lib.PI32),
                                     None if mat is None else mat.ctypes.data_as(_lib.PI32)), "ep_sim_upload_mesh")

    def set_region(self, region: int, variant=None, params=None, sigma=None, conductive=True, model=None):
        """ep_sim_set_region: cell type (name or EP_CELL_*; None: the sim's),
        positional parameter overrides, conductivities (l, t, n) in mS/mm
        (None: the sim's) and whether the subdomain conducts; model: the
        subdomain's ionic model ("ap", "bo", "ttp06", "passive"; None: the
        sim's), ep_sim_set_region_model."""
        if model is not None:
            check(lib.ep_sim_set_region_model(self._h, int(region), MODEL_IDS[model]), "ep_sim_set_region_model")
        v = -1 if variant is None else (CELL_IDS[variant] if isinstance(variant, str) else int(variant))
        p = None if params is None or len(params) == 0 else _f64(params)
        sl, st, sn = (-1.0, -1.0, -1.0) if sigma is None else tuple(float(x) for x in sigma)
        check(lib.ep_sim_set_region(self._h, int(region), v, _pd(p) if p is not None else None,
                                    0 if p is None else p.size, sl, st, sn, 1 if conductive else 0),
              "ep_sim_set_region")

    def upload_fibers(self, f0, s0, n0):
        f0, s0, n0 = _f64(f0), _f64(s0), _f64(n0)
        check(lib.ep_sim_upload_fibers(self._h, _pd(f0), _pd(s0), _pd(n0)), "ep_sim_upload_fibers")

    def set_conductivity(self, sigma_l, sigma_t, sigma_n, chi, cm):
        check(lib.ep_sim_set_conductivity(self._h, sigma_l, sigma_t, sigma_n, chi, cm),
              "ep_sim_set_conductivity")

    def set_ionic_model(self, model: int, variant: int = 0, params=None, init_state=None):
        p = _f64(params) if params is not None else None
        s = _f64(init_state) if init_state is not None else None
        check(lib.ep_sim_set_ionic_model(self._h, int(model), int(variant), _pd(p) if p is not None else None,
                                         0 if p is None else p.size, _pd(s) if s is not None else None),
              "ep_sim_set_ionic_model")

    def add_stimulus(self, shape, center, size, amp, t0=0.0, dur=2.0, period=0.0):
        c = _f64(center)
        check(lib.ep_sim_add_stimulus(self._h, int(shape), _pd(c), size, amp, t0, dur, period),
              "ep_sim_add_stimulus")

    def set_solver(self, dt, bdf=1, precision=EP_FP64, precond=EP_JACOBI, block=1, rtol=1e-10, max_it=1000):
        self.bdf = int(bdf)
        check(lib.ep_sim_set_solver(self._h, dt, int(bdf), int(precision), int(precond), int(block), rtol,
                                    int(max_it)), "ep_sim_set_solver")

    def set_option(self, key, value):
        check(lib.ep_sim_set_option(self._h, int(key), float(value)), "ep_sim_set_option")

    def autotune(self, trial_steps: int = 10):
        """Launch-shape tuner (advances the simulation by 5 * trial_steps
        steps); returns (ionic nodes per thread, tile map)."""
        a, b = C.c_int32(), C.c_int32()
        check(lib.ep_sim_autotune(self._h, int(trial_steps), C.byref(a), C.byref(b)), "ep_sim_autotune")
        return a.value, b.value

    def finalize(self):
        check(lib.ep_sim_finalize(self._h), "ep_sim_finalize")

    def device_bytes_estimate(self) -> int:
        v = C.c_size_t()
        check(lib.ep_sim_device_bytes_estimate(self._h, C.byref(v)), "ep_sim_device_bytes_estimate")
        return int(v.value)

    # -- stepping and results ---------------------------------------------------
    def step(self, n_steps: int = 1, allow_noconv: bool = False):
        return check(lib.ep_sim_step(self._h, int(n_steps)), "ep_sim_step",
                     allow=(_lib.EP_ENOCONV,) if allow_noconv else ())

    def sync(self):
        check(lib.ep_sim_sync(self._h), "ep_sim_sync")

    def get_potential(self):
        out = np.empty(self.n_nodes)
        check(lib.ep_sim_get_potential(self._h, _pd(out)), "ep_sim_get_potential")
        return out

    def get_potential_device(self, dst_ptr: int, dtype: int = EP_DTYPE_F64):
        check(lib.ep_sim_get_potential_device(self._h, C.c_void_p(dst_ptr), int(dtype)),
              "ep_sim_get_potential_device")

    def get_activation_times(self):
        out = np.empty(self.n_nodes)
        check(lib.ep_sim_get_activation_times(self._h, _pd(out)), "ep_sim_get_activation_times")
        return out

    def get_threshold_times(self):
        out = np.empty(self.n_nodes)
        check(lib.ep_sim_get_threshold_times(self._h, _pd(out)), "ep_sim_get_threshold_times")
        return out

    def get_stats(self) -> dict:
        st = EpStats()
        check(lib.ep_sim_get_stats(self._h, C.byref(st)), "ep_sim_get_stats")
        return {name: getattr(st, name) for name, _ in EpStats._fields_}

    def timer_overhead_us(self, reps: int = 200) -> float:
        """Mean duration of an empty HIP event pair on the sim's stream (us)."""
        v = C.c_double()
        check(lib.ep_sim_timer_overhead(self._h, int(reps), C.byref(v)), "ep_sim_timer_overhead")
        return v.value

    def time_kernel_us(self, kind: str, reps: int = 200) -> float:
        """ep_sim_time_kernel for "cg_spmv", "rhs" or "cg_pipe" (between steps)."""
        v = C.c_double()
        check(lib.ep_sim_time_kernel(self._h, KERNEL_KINDS.index(kind), int(reps), C.byref(v)),
              "ep_sim_time_kernel")
        return v.value

    def get_kernel_times(self) -> dict:
        ms = np.zeros(len(KERNEL_KINDS))
        cnt = np.zeros(len(KERNEL_KINDS), np.int64)
        check(lib.ep_sim_get_kernel_times(self._h, _pd(ms), cnt.ctypes.data_as(_lib.PI64)),
              "ep_sim_get_kernel_times")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_KINDS)}

    @property
    def n_vars(self) -> int:
        return lib.ep_sim_n_vars(self._h)

    def set_state(self, u, w, u_prev=None, step_index: int = 0):
        u = _f64(u)
        w = _f64(w, (self.n_vars, self.n_nodes)) if self.n_vars else np.zeros(1)
        up = _f64(u_prev) if u_prev is not None else None
        check(lib.ep_sim_set_state(self._h, _pd(u), _pd(w), _pd(up) if up is not None else None,
                                   int(step_index)), "ep_sim_set_state")

    def get_state(self):
        u = np.empty(self.n_nodes)
        w = np.empty((max(self.n_vars, 0), self.n_nodes))
        up = np.empty((max(self.bdf - 1, 1), self.n_nodes))
        check(lib.ep_sim_get_state(self._h, _pd(u), _pd(w) if self.n_vars else None, _pd(up)),
              "ep_sim_get_state")
        return u, w, up[: self.bdf - 1]

    def close(self):
        if getattr(self, "_h", None):
            lib.ep_sim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- convenience -----------------------------------------------------------
    @classmethod
    def from_spec(cls, spec, precision=EP_FP64, device=0, stream=None, rtol=None, max_it=1000,
                  matrix_format=EP_FMT_AUTO, finalize=True, inner_rtol=None, block=1, ionic_scheme="rl",
                  material=None, regions=None, ionic_fp64=False, cg_variant=EP_CG_AUTO,
                  initial_guess=EP_X0_EXT):
        """Configure from a workloads.SimSpec (marshalling of its arrays).
        block > 1 selects block-Jacobi preconditioning with that block size;
        ionic_fp64: in mixed precision, step the ionic model in FP64;
        ionic_scheme "rl" (Rush-Larsen) or "bdf" (the paper's semi-implicit
        BDF).  material: per-element subdomain labels; regions: {label:
        dict(variant=, params=, sigma=, conductive=)} passed to set_region;
        cg_variant: the CG formulation (EP_CG_*); initial_guess: EP_X0_*."""
        sim = cls(device, stream)
        m = spec.mesh
        sim.upload_mesh(m.elem, m.xyz, m.conn, material)
        for r, cfg in (regions or {}).items():
            sim.set_region(r, **cfg)
        if spec.fibers is not None:
            sim.upload_fibers(*spec.fibers)
        p = spec.phys
        sim.set_conductivity(p.sigma_l, p.sigma_t, p.sigma_n, p.chi, p.cm)
        sim.set_ionic_model(MODEL_IDS[spec.model], CELL_IDS.get(spec.variant, 0))
        for st in spec.stimuli:
            sim.add_stimulus(st.shape, st.center, st.size, st.amp, st.t0, st.dur, st.period)
        sim.set_solver(spec.dt, spec.bdf, precision, EP_BJACOBI if block > 1 else EP_JACOBI, int(block),
                       spec.rtol if rtol is None else rtol, max_it)
        if matrix_format != EP_FMT_AUTO:
            sim.set_option(EP_OPT_MATRIX_FORMAT, matrix_format)
        if inner_rtol is not None:
            sim.set_option(EP_OPT_INNER_RTOL, inner_rtol)
        if ionic_scheme != "rl":
            sim.set_option(EP_OPT_IONIC_SCHEME, {"bdf": EP_IONIC_BDF}[ionic_scheme])
        if ionic_fp64:
            sim.set_option(EP_OPT_IONIC_FP64, 1)
        if cg_variant != EP_CG_AUTO:
            sim.set_option(EP_OPT_CG_VARIANT, cg_variant)
        if initial_guess != EP_X0_EXT:
            sim.set_option(EP_OPT_INITIAL_GUESS, initial_guess)
        if finalize:
            sim.finalize()
        return sim


class Pool:
    """Batched / serving container of resident simulations (wraps ep_pool)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int, precision: int = EP_FP64, device: int = 0,
                 stream=None):
        h = C.c_void_p()
        check(lib.ep_pool_create(int(device), C.c_void_p(stream) if stream else None, int(hbm_budget_bytes),
                                 int(max_slots), int(precision), C.byref(h)), "ep_pool_create")
        self._h = h
        self.sims = {}

    def admit(self, sim: "Simulation", n_steps_total: int):
        """Slot id, or None when the pool is full (EP_EAGAIN)."""
        slot = C.c_int32()
        st = check(lib.ep_pool_admit(self._h, sim._h, int(n_steps_total), C.byref(slot)), "ep_pool_admit",
                   allow=(_lib.EP_EAGAIN,))
        if st == _lib.EP_EAGAIN:
            return None
        self.sims[slot.value] = sim
        return slot.value

    def step(self, n_steps: int = 1):
        check(lib.ep_pool_step(self._h, int(n_steps)), "ep_pool_step")

    def poll(self):
        cap = max(1, len(self.sims))
        buf = np.zeros(cap, np.int32)
        n = C.c_int32()
        check(lib.ep_pool_poll(self._h, buf.ctypes.data_as(_lib.PI32), cap, C.byref(n)), "ep_pool_poll")
        return [int(x) for x in buf[: n.value]]

    def release(self, slot: int, allow_error: bool = False):
        """Remove a slot; returns (sim, status)."""
        out = C.c_void_p()
        st = check(lib.ep_pool_release(self._h, int(slot), C.byref(out)), "ep_pool_release",
                   allow=(_lib.EP_ENAN, _lib.EP_ENOCONV) if allow_error else ())
        return self.sims.pop(slot), st

    def set_option(self, key, value):
        check(lib.ep_pool_set_option(self._h, int(key), float(value)), "ep_pool_set_option")

    def autotune(self, trial_steps: int = 10):
        """ep_pool_autotune; returns (ionic nodes per thread, tile map)."""
        a, b = C.c_int32(), C.c_int32()
        check(lib.ep_pool_autotune(self._h, int(trial_steps), C.byref(a), C.byref(b)), "ep_pool_autotune")
        return a.value, b.value

    def info(self):
        a = C.c_int32()
        b = C.c_size_t()
        check(lib.ep_pool_get_info(self._h, C.byref(a), C.byref(b)), "ep_pool_get_info")
        return {"active": a.value, "bytes_in_use": b.value}

    def close(self):
        if getattr(self, "_h", None):
            lib.ep_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cell_pace(model, variant="", n_cells=1, params=None, init=None, dt=0.05, bdf=2, period=800.0,
              stim_mV_per_ms=40.0, stim_dur=1.0, n_beats=1, device=0):
    """ep_cell_pace: pace single cells on the GPU; returns [n_cells, 1 + n_vars]
    (u, then the state), each row usable as an initial state."""
    mid = MODEL_IDS[model]
    nv = {EP_PASSIVE: 0, EP_AP: 1, EP_BO: 3, EP_TTP06: 18}[mid]
    out = np.zeros((int(n_cells), 1 + nv))
    p = None if params is None else _f64(np.atleast_2d(params))
    ini = None if init is None else _f64(np.atleast_2d(init))
    check(lib.ep_cell_pace(int(device), mid, CELL_IDS.get(variant, 0), int(n_cells), _pd(p) if p is not None else None,
                           0 if p is None else int(p.shape[1]), _pd(ini) if ini is not None else None, float(dt),
                           int(bdf), float(period), float(stim_mV_per_ms), float(stim_dur), int(n_beats), _pd(out)),
          "ep_cell_pace")
    return out


def cell_pace_device(model, variant="", n_cells=1, params_ptr=0, n_params=0, init_ptr=0, out_ptr=0, dt=0.05,
                     bdf=2, period=800.0, stim_mV_per_ms=40.0, stim_dur=1.0, n_beats=1, device=0, stream=0):
    """ep_cell_pace_device: ep_cell_pace on caller-owned device buffers (raw
    device addresses, e.g. torch tensors' data_ptr()), enqueued on `stream`
    without allocating or synchronizing."""
    check(lib.ep_cell_pace_device(int(device), C.c_void_p(stream) if stream else None, MODEL_IDS[model],
                                  CELL_IDS.get(variant, 0), int(n_cells),
                                  C.c_void_p(params_ptr) if params_ptr else None, int(n_params),
                                  C.c_void_p(init_ptr) if init_ptr else None, float(dt), int(bdf), float(period),
                                  float(stim_mV_per_ms), float(stim_dur), int(n_beats), C.c_void_p(out_ptr)),
          "ep_cell_pace_device")


def assemble_csr(elem, xyz, conn, fibers=None, sigma=(0.17, 0.019, 0.019), chi=140.0, cm=0.01):
    """The library's host-side FE assembly (ep_assemble_csr): (rowptr, col, valM, valK)."""
    xyz = _f64(xyz)
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    if fibers is not None:
        f0, s0, n0 = (_f64(a) for a in fibers)
        fp = (_pd(f0), _pd(s0), _pd(n0))
    else:
        fp = (None, None, None)
    nnz = C.c_int64()
    args = (int(elem), xyz.shape[0], _pd(xyz), conn.shape[0], conn.ctypes.data_as(_lib.PI32), *fp,
            sigma[0], sigma[1], sigma[2], chi, cm)
    check(lib.ep_assemble_csr(*args, C.byref(nnz), None, None, None, None), "ep_assemble_csr")
    rowptr = np.empty(xyz.shape[0] + 1, np.int64)
    col = np.empty(nnz.value, np.int32)
    vm = np.empty(nnz.value)
    vk = np.empty(nnz.value)
    check(lib.ep_assemble_csr(*args, C.byref(nnz), rowptr.ctypes.data_as(_lib.PI64),
                              col.ctypes.data_as(_lib.PI32), _pd(vm), _pd(vk)), "ep_assemble_csr")
    return rowptr, col, vm, vk


def version() -> str:
    return lib.ep_version().decode()
