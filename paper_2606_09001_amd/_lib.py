"""ctypes declarations of libamg355.so (the C ABI in include/amg355.h).

Argument marshalling only: every step of setup and solve runs in the HIP
library.  Importing this module fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamg355.so")

AMG_OK = 0
AMG_NOT_CONVERGED = 1
AMG_ERR_INVALID_ARG = -1
AMG_ERR_ZERO_DIAG = -2
AMG_ERR_PATTERN_MISMATCH = -3
AMG_ERR_BREAKDOWN = -4
AMG_ERR_OOM = -5
AMG_ERR_HIP = -6
AMG_ERR_COARSE_TOO_LARGE = -7
AMG_ERR_SCRATCH_LIMIT = -8
AMG_NOALLOC_MAX_N = 2097152
AMG_MAX_DENSE_COARSE = 2048

AMG_PREC_FP64 = 0
AMG_PREC_FP32 = 1
AMG_SMOOTHER_JACOBI = 0
AMG_SMOOTHER_L1 = 1
AMG_SOLVER_PCG = 0
AMG_SOLVER_BICGSTAB = 1
AMG_MAX_LEVELS = 20

FIELDS = {
    "agg": 0, "A_rp": 1, "A_ci": 2, "A_v": 3, "A_v32": 4, "dinv": 5, "P_rp": 6, "P_ci": 7, "P_v": 8,
    "P_bf16": 9, "R_rp": 10, "R_ci": 11, "R_v": 12, "R_bf16": 13, "G_rp": 14, "G_ci": 15,
    "coarse_factor": 16, "coarse_inv": 17, "sw32": 18, "coarse_pivots": 19, "sw": 20, "coarse_inv32": 21,
}

EXPORTS = [
    "amg_params_default", "amg_setup", "amg_update_values", "amg_solve", "amg_solve_adjoint", "amg_pattern_grad",
    "amg_apply_vcycle", "amg_hierarchy_stats", "amg_field_info", "amg_export_field", "amg_destroy", "amg_finalize",
    "amg_cache_size", "amg_set_cache_capacity", "amg_status_string", "amg_instrument", "amg_instrument_read",
    "amg_kernel_bytes", "amg_pattern_grad_batched", "amg_solve_columns", "amg_color_columns",
    "amg_probe_vectors", "amg_probe_assemble", "amg_probe_scatter", "amg_convert_bf16", "amg_solve_noalloc",
    "amg_kernel_bytes_batched",
]

KERNELS = {"spmv_dot": 0, "pre": 1, "post": 2, "restrict": 3, "prolong": 4, "cg_update": 5, "xpay": 6, "coarse": 7}


class amg_params(C.Structure):
    _fields_ = [
        ("vcycle_prec", C.c_int), ("transfer_bf16", C.c_int), ("theta", C.c_double), ("max_coarse", C.c_int),
        ("max_levels", C.c_int), ("smoother", C.c_int), ("omega", C.c_double), ("nu_pre", C.c_int),
        ("nu_post", C.c_int), ("maxiter", C.c_int), ("flexible", C.c_int), ("symmetric", C.c_int),
        ("check_every", C.c_int), ("use_graphs", C.c_int), ("autotune", C.c_int), ("precondition", C.c_int),
        ("solver", C.c_int), ("fused_small", C.c_int),
    ]


class amg_info(C.Structure):
    _fields_ = [
        ("iters", C.c_int), ("rel_resid", C.c_double), ("status", C.c_int), ("cache_event", C.c_int),
        ("restarts", C.c_int), ("setup_ms", C.c_double), ("solve_ms", C.c_double),
    ]

    def to_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_L20 = C.c_int64 * AMG_MAX_LEVELS
_D20 = C.c_double * AMG_MAX_LEVELS
_I20 = C.c_int * AMG_MAX_LEVELS


class amg_hier_stats(C.Structure):
    _fields_ = [
        ("num_levels", C.c_int), ("n", _L20), ("nnz", _L20), ("nnz_p", _L20), ("nnz_g", _L20), ("rho", _D20),
        ("omega_p", _D20), ("mis_rounds", _I20), ("operator_complexity", C.c_double), ("group_a", _I20),
        ("group_p", _I20), ("group_r", _I20), ("form_a", _I20), ("sliced_len", _L20),
        ("single_workgroup", C.c_int),
    ]

    def to_dict(self):
        L = self.num_levels
        d = {"num_levels": L, "operator_complexity": self.operator_complexity,
             "single_workgroup": self.single_workgroup}
        for f in ("n", "nnz", "nnz_p", "nnz_g", "rho", "omega_p", "mis_rounds", "group_a", "group_p", "group_r",
                  "form_a", "sliced_len"):
            d[f] = list(getattr(self, f))[:L]
        return d


_lib = None


def load():
    """Load libamg355.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          f"`python -m paper_2606_09001_amd.csrc.build` (or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.amg_params_default.argtypes = [C.POINTER(amg_params)]
    L.amg_params_default.restype = None
    L.amg_setup.argtypes = [C.POINTER(amg_params), i32, i64, vp, vp, vp, i32, vp, C.POINTER(vp)]
    L.amg_update_values.argtypes = [vp, vp, vp]
    L.amg_solve.argtypes = [vp, vp, vp, dbl, i32, C.POINTER(amg_info), vp]
    L.amg_solve_noalloc.argtypes = [vp, vp, vp, dbl, C.POINTER(amg_info), vp]
    L.amg_solve_adjoint.argtypes = [vp, vp, vp, dbl, i32, C.POINTER(amg_info), vp]
    L.amg_pattern_grad.argtypes = [vp, vp, vp, vp, vp]
    L.amg_apply_vcycle.argtypes = [vp, vp, vp, vp]
    L.amg_hierarchy_stats.argtypes = [vp, C.POINTER(amg_hier_stats)]
    L.amg_field_info.argtypes = [vp, C.c_int, C.c_int, C.POINTER(i64), C.POINTER(C.c_int)]
    L.amg_export_field.argtypes = [vp, C.c_int, C.c_int, vp, C.c_size_t, vp]
    L.amg_destroy.argtypes = [vp]
    L.amg_finalize.argtypes = []
    L.amg_cache_size.argtypes = []
    L.amg_cache_size.restype = C.c_int
    L.amg_set_cache_capacity.argtypes = [C.c_int]
    L.amg_instrument.argtypes = [vp, C.c_int, C.c_int]
    L.amg_instrument_read.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(dbl), C.POINTER(dbl), C.POINTER(dbl)]
    L.amg_kernel_bytes.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.POINTER(dbl)]
    L.amg_kernel_bytes_batched.argtypes = [vp, C.c_int, C.c_int, C.c_int, i32, C.POINTER(dbl)]
    L.amg_pattern_grad_batched.argtypes = [vp, vp, vp, i32, vp, vp]
    L.amg_solve_columns.argtypes = [vp, i32, vp, vp, vp]
    L.amg_color_columns.argtypes = [i32, i64, vp, vp, vp, C.POINTER(i32), vp]
    L.amg_probe_vectors.argtypes = [i32, vp, i32, vp, vp]
    L.amg_probe_assemble.argtypes = [i32, i64, vp, vp, vp, i32, vp, vp, vp]
    L.amg_probe_scatter.argtypes = [i32, i64, vp, vp, vp, i32, vp, vp, vp]
    L.amg_convert_bf16.argtypes = [vp, vp, i64, vp]
    L.amg_status_string.argtypes = [C.c_int]
    L.amg_status_string.restype = C.c_char_p
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("amg_params_default", "amg_cache_size", "amg_status_string"):
            f.restype = C.c_int
    _lib = L
    return L


def status_string(st: int) -> str:
    return load().amg_status_string(st).decode()


class AmgError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status_string(status)} ({status})")
        self.status = status


def check(st: int, where: str, allow=(AMG_OK,)):
    if st not in allow:
        raise AmgError(st, where)
    return st
