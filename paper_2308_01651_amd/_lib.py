"""ctypes declarations of libep_mi355x.so (the C ABI in include/ep.h).

Argument marshalling only.  Importing this module loads the HIP library and
fails loudly if it has not been built; nothing here computes any part of the
time step.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libep_mi355x.so")

EP_OK, EP_EINVAL, EP_ENOMEM, EP_EHIP, EP_ENOCONV, EP_ENAN, EP_EAGAIN, EP_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "EP_OK", -1: "EP_EINVAL", -2: "EP_ENOMEM", -3: "EP_EHIP", -4: "EP_ENOCONV",
                -5: "EP_ENAN", -6: "EP_EAGAIN", -7: "EP_ESTATE"}


class EpError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class EpStats(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("nnz", C.c_int64), ("steps", C.c_int64),
                ("cg_iters_total", C.c_int64), ("cg_iters_last", C.c_int32),
                ("cg_iters_max", C.c_int32), ("ir_sweeps_total", C.c_int64),
                ("rel_residual_last", C.c_double), ("matrix_format", C.c_int32),
                ("n_diag", C.c_int32), ("device_bytes", C.c_int64), ("ms_ionic", C.c_double),
                ("ms_rhs", C.c_double), ("ms_solve", C.c_double), ("ms_activation", C.c_double),
                ("ms_setup", C.c_double), ("mf_compressed", C.c_int32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                      "(python paper_2308_01651_amd/build.py)")

# PyTorch ships its own HIP runtime with the same soname as the system one.
# Loading torch first makes this library bind to that runtime, so that one
# process holds a single HIP runtime and torch tensors / streams interoperate.
try:
    import torch  # noqa: F401
except ImportError:  # torch is optional for the C ABI itself
    torch = None

lib = C.CDLL(LIB_PATH)

P = C.c_void_p
PD = C.POINTER(C.c_double)
PI32 = C.POINTER(C.c_int32)
PI64 = C.POINTER(C.c_int64)
PP = C.POINTER(C.c_void_p)

_SIGS = {
    "ep_sim_create": [C.c_int, P, PP],
    "ep_sim_upload_mesh": [P, C.c_int, C.c_int64, PD, C.c_int64, PI32, PI32],
    "ep_sim_upload_fibers": [P, PD, PD, PD],
    "ep_sim_set_conductivity": [P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double],
    "ep_sim_set_ionic_model": [P, C.c_int, C.c_int, PD, C.c_int, PD],
    "ep_sim_set_region": [P, C.c_int, C.c_int, PD, C.c_int, C.c_double, C.c_double, C.c_double, C.c_int],
    "ep_sim_add_stimulus": [P, C.c_int, PD, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double],
    "ep_sim_set_solver": [P, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int],
    "ep_sim_set_option": [P, C.c_int, C.c_double],
    "ep_sim_finalize": [P],
    "ep_sim_step": [P, C.c_int],
    "ep_sim_sync": [P],
    "ep_sim_get_potential": [P, PD],
    "ep_sim_get_potential_device": [P, P, C.c_int],
    "ep_sim_get_activation_times": [P, PD],
    "ep_sim_get_threshold_times": [P, PD],
    "ep_sim_get_stats": [P, C.POINTER(EpStats)],
    "ep_sim_get_kernel_times": [P, PD, PI64],
    "ep_sim_set_state": [P, PD, PD, PD, C.c_int64],
    "ep_sim_get_state": [P, PD, PD, PD],
    "ep_sim_device_bytes_estimate": [P, C.POINTER(C.c_size_t)],
    "ep_pool_create": [C.c_int, P, C.c_size_t, C.c_int, C.c_int, PP],
    "ep_pool_admit": [P, P, C.c_int64, PI32],
    "ep_pool_step": [P, C.c_int],
    "ep_pool_poll": [P, PI32, C.c_int, PI32],
    "ep_pool_release": [P, C.c_int, PP],
    "ep_pool_get_info": [P, PI32, C.POINTER(C.c_size_t)],
    "ep_pool_set_option": [P, C.c_int, C.c_double],
    "ep_pool_autotune": [P, C.c_int, PI32, PI32],
    "ep_sim_autotune": [P, C.c_int, PI32, PI32],
    "ep_sim_timer_overhead": [P, C.c_int, PD],
    "ep_sim_time_kernel": [P, C.c_int, C.c_int, PD],
    "ep_cell_pace": [C.c_int, C.c_int, C.c_int, C.c_int, PD, C.c_int, PD, C.c_double, C.c_int, C.c_double,
                     C.c_double, C.c_double, C.c_int, PD],
    "ep_sim_set_region_model": [P, C.c_int, C.c_int],
    "ep_cell_pace_device": [C.c_int, P, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_double,
                            C.c_int, C.c_double, C.c_double, C.c_double, C.c_int, C.c_void_p],
    "ep_assemble_csr": [C.c_int, C.c_int64, PD, C.c_int64, PI32, PD, PD, PD, C.c_double, C.c_double,
                        C.c_double, C.c_double, C.c_double, PI64, PI64, PI32, PD, PD],
}
for _name, _args in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int

lib.ep_sim_destroy.argtypes = [P]
lib.ep_sim_destroy.restype = None
lib.ep_pool_destroy.argtypes = [P]
lib.ep_pool_destroy.restype = None
lib.ep_sim_n_vars.argtypes = [P]
lib.ep_sim_n_vars.restype = C.c_int
lib.ep_last_error.argtypes = []
lib.ep_last_error.restype = C.c_char_p
lib.ep_version.argtypes = []
lib.ep_version.restype = C.c_char_p


def check(status: int, where: str, allow=()):
    if status != EP_OK and status not in allow:
        raise EpError(status, where, lib.ep_last_error().decode(errors="replace"))
    return status


def exported_names():
    """Names the header declares; used by the symbol-export test."""
    return sorted(_SIGS) + ["ep_sim_destroy", "ep_pool_destroy", "ep_sim_n_vars", "ep_last_error",
                            "ep_version"]
