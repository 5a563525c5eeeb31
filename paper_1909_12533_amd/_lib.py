"""ctypes declarations of the C ABI in ``include/sp2dm.h``."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsp2dm.so")

SP2_OK = 0
SP2_ERR_INVALID_ARG = -1
SP2_ERR_BAD_BOUNDS = -2
SP2_ERR_NONFINITE = -3
SP2_ERR_OOM = -4
SP2_ERR_HIP = -5
SP2_WARN_NOT_CONVERGED = 1
SP2_WARN_TRACE = 2

PREC_FP64, PREC_FP32, PREC_BF16X3 = 0, 1, 2
TRUNC_NONE, TRUNC_FROB, TRUNC_FROBINF = 0, 1, 2
STOP_CRITERION, STOP_IDEMPOTENCY, STOP_NMAX, STOP_NOISE_FLOOR = 1, 2, 3, 4

# names of every exported entry point declared in include/sp2dm.h
EXPORTS = [
    "sp2_version", "sp2_options_default", "sp2_create", "sp2_destroy", "sp2_set_allocator", "sp2_trim",
    "sp2_last_error", "sp2_gershgorin", "sp2_density", "sp2_vjp", "sp2_jvp", "sp2_replay", "sp2_tape_info",
    "sp2_square_step", "sp2_truncate", "sp2_bsr_copy", "sp2_bsr_free", "sp2_tape_free", "sp2_schedule",
    "sp2_homo_lumo", "sp2_pair_product", "sp2_matrix_norms", "sp2_density_begin", "sp2_density_step",
    "sp2_density_end", "sp2_solver_free", "sp2_matrix_norms_noalloc", "sp2_general_from_upper",
    "sp2_general_product",
]


class sp2_bsr(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("bs", C.c_int32),
        ("owned", C.c_int32),
        ("nbr", C.c_int64),
        ("nnzb", C.c_int64),
        ("row_ptr", C.c_void_p),
        ("col_idx", C.c_void_p),
        ("val", C.c_void_p),
    ]


class sp2_options(C.Structure):
    _fields_ = [
        ("accel", C.c_int32),
        ("precision", C.c_int32),
        ("switch_tol", C.c_double),
        ("trunc_norm", C.c_int32),
        ("n_max_cap", C.c_int32),
        ("coarse_bs", C.c_int64),
        ("gamma", C.c_double),
        ("tau_fixed", C.c_double),
        ("idem_stop", C.c_double),
        ("record_tape", C.c_int32),
        ("n_checkpoints", C.c_int32),
        ("correct", C.c_int32),
        ("corr_purify", C.c_int32),
        ("corr_tol", C.c_double),
        ("corr_mem", C.c_int64),
        ("adjoint_precision", C.c_int32),
        ("corr_deriv_tol", C.c_double),
        ("corr_mcweeny", C.c_int32),
        ("corr_host_mem", C.c_int64),
        ("low_start_xi", C.c_double),
        ("tail_storage", C.c_int32),
        ("low_floor_stop", C.c_int32),
    ]


_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int32)
_LP = C.POINTER(C.c_int64)


class sp2_stats(C.Structure):
    _fields_ = [
        ("capacity", C.c_int32),
        ("n_iter", C.c_int32),
        ("n_max", C.c_int32),
        ("n_min", C.c_int32),
        ("stop_reason", C.c_int32),
        ("switch_iter", C.c_int32),
        ("homo_ub_est", C.c_double),
        ("lumo_lb_est", C.c_double),
        ("subspace_err_bound", C.c_double),
        ("time_s", C.c_double),
        ("alg_flops", C.c_double),
        ("max_nnzb", C.c_int64),
        ("e", _DP),
        ("t", _DP),
        ("trace", _DP),
        ("alpha", _DP),
        ("tau", _DP),
        ("trunc_err_frob", _DP),
        ("trunc_err_mixed", _DP),
        ("iter_time_s", _DP),
        ("iter_flops", _DP),
        ("p", _IP),
        ("precision", _IP),
        ("nnzb", _LP),
        ("square_time_s", _DP),
        ("square_time_total_s", C.c_double),
        ("corr_rounds", C.c_int32),
        ("corr_time_s", C.c_double),
        ("corr_flops", C.c_double),
        ("corr_delta_norm", C.c_double),
        ("corr_step_norm", C.c_double),
        ("corr_e_last", C.c_double),
        ("corr_max_nnzb", C.c_int64),
        ("seq_bytes", C.c_int64),
        ("seq_host_bytes", C.c_int64),
        ("corr_recomputed", C.c_int32),
        ("device_peak_bytes", C.c_int64),
    ]


STEP_ITERATION, STEP_CORRECTION = 1, 2


class sp2_step_info(C.Structure):
    _fields_ = [
        ("done", C.c_int32),
        ("kind", C.c_int32),
        ("iteration", C.c_int32),
        ("precision", C.c_int32),
        ("flops", C.c_double),
        ("wall_s", C.c_double),
        ("kernel_s", C.c_double * 3),
        ("kernel_flops", C.c_double * 3),
        ("kernel_launches", C.c_int32 * 3),
    ]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"HIP library {path} is missing: build it first (python -m paper_1909_12533_amd.build)")
    lib = C.CDLL(path)
    P = C.POINTER
    lib.sp2_version.restype = C.c_char_p
    lib.sp2_version.argtypes = []
    lib.sp2_options_default.restype = None
    lib.sp2_options_default.argtypes = [P(sp2_options)]
    lib.sp2_create.restype = C.c_int
    lib.sp2_create.argtypes = [P(C.c_void_p), C.c_int, C.c_void_p]
    lib.sp2_destroy.restype = None
    lib.sp2_destroy.argtypes = [C.c_void_p]
    lib.sp2_set_allocator.restype = C.c_int
    lib.sp2_set_allocator.argtypes = [C.c_void_p, ALLOC_FN, FREE_FN, C.c_void_p]
    lib.sp2_trim.restype = None
    lib.sp2_trim.argtypes = [C.c_void_p]
    lib.sp2_last_error.restype = C.c_char_p
    lib.sp2_last_error.argtypes = [C.c_void_p]
    lib.sp2_gershgorin.restype = C.c_int
    lib.sp2_gershgorin.argtypes = [C.c_void_p, P(sp2_bsr), P(C.c_double), P(C.c_double)]
    lib.sp2_density.restype = C.c_int
    lib.sp2_density.argtypes = [C.c_void_p, P(sp2_bsr), C.c_int64, C.c_double, C.c_double, P(C.c_double),
                                P(C.c_double), P(sp2_options), P(P(sp2_bsr)), P(C.c_double), P(C.c_double),
                                P(sp2_stats), P(C.c_void_p)]
    lib.sp2_density_begin.restype = C.c_int
    lib.sp2_density_begin.argtypes = [C.c_void_p, P(sp2_bsr), C.c_int64, C.c_double, C.c_double, P(C.c_double),
                                      P(C.c_double), P(sp2_options), P(C.c_void_p)]
    lib.sp2_density_step.restype = C.c_int
    lib.sp2_density_step.argtypes = [C.c_void_p, C.c_void_p, P(sp2_step_info)]
    lib.sp2_density_end.restype = C.c_int
    lib.sp2_density_end.argtypes = [C.c_void_p, C.c_void_p, P(P(sp2_bsr)), P(C.c_double), P(C.c_double),
                                    P(sp2_stats), P(C.c_void_p)]
    lib.sp2_solver_free.restype = None
    lib.sp2_solver_free.argtypes = [C.c_void_p, C.c_void_p]
    for name in ("sp2_vjp", "sp2_jvp", "sp2_replay"):
        f = getattr(lib, name)
        f.restype = C.c_int
        f.argtypes = [C.c_void_p, C.c_void_p, P(sp2_bsr), P(P(sp2_bsr))]
    lib.sp2_tape_info.restype = C.c_int
    lib.sp2_tape_info.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_int32), P(C.c_int64)]
    lib.sp2_square_step.restype = C.c_int
    lib.sp2_square_step.argtypes = [C.c_void_p, P(sp2_bsr), C.c_double, C.c_double, C.c_double, C.c_int,
                                    P(P(sp2_bsr)), P(C.c_double)]
    lib.sp2_pair_product.restype = C.c_int
    lib.sp2_pair_product.argtypes = [C.c_void_p, P(sp2_bsr), P(sp2_bsr), P(sp2_bsr), C.c_int, C.c_int, C.c_double,
                                     C.c_double, C.c_double, C.c_int, P(P(sp2_bsr)), P(C.c_double)]
    lib.sp2_general_from_upper.restype = C.c_int
    lib.sp2_general_from_upper.argtypes = [C.c_void_p, P(sp2_bsr), P(P(sp2_bsr))]
    lib.sp2_general_product.restype = C.c_int
    lib.sp2_general_product.argtypes = [C.c_void_p, P(sp2_bsr), P(sp2_bsr), P(sp2_bsr), C.c_double, C.c_double,
                                        C.c_double, C.c_int, P(P(sp2_bsr)), P(C.c_double)]
    lib.sp2_truncate.restype = C.c_int
    lib.sp2_truncate.argtypes = [C.c_void_p, P(sp2_bsr), C.c_double, C.c_int, C.c_int64, P(P(sp2_bsr)),
                                 P(C.c_double)]
    lib.sp2_matrix_norms.restype = C.c_int
    lib.sp2_matrix_norms.argtypes = [C.c_void_p, P(sp2_bsr), C.c_int64, P(C.c_double), P(C.c_double)]
    lib.sp2_matrix_norms_noalloc.restype = C.c_int
    lib.sp2_matrix_norms_noalloc.argtypes = [C.c_void_p, P(sp2_bsr), C.c_int64, P(C.c_double), P(C.c_double)]
    lib.sp2_bsr_copy.restype = C.c_int
    lib.sp2_bsr_copy.argtypes = [C.c_void_p, P(sp2_bsr), C.c_void_p, C.c_void_p, C.c_void_p]
    lib.sp2_bsr_free.restype = None
    lib.sp2_bsr_free.argtypes = [C.c_void_p, P(sp2_bsr)]
    DP, IP = P(C.c_double), P(C.c_int32)
    lib.sp2_schedule.restype = C.c_int
    lib.sp2_schedule.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, C.c_double, C.c_double,
                                 C.c_int, IP, IP, IP, DP, DP, DP, DP, DP]
    lib.sp2_homo_lumo.restype = C.c_int
    lib.sp2_homo_lumo.argtypes = [C.c_int, C.c_int, DP, DP, IP, DP, DP, DP, C.c_double, C.c_double, C.c_int64,
                                  C.c_int64, DP, DP]
    lib.sp2_tape_free.restype = None
    lib.sp2_tape_free.argtypes = [C.c_void_p, C.c_void_p]
    _lib = lib
    return lib
