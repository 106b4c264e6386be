"""ctypes loader for libmr1l.so (argument marshalling only; every step runs in the HIP library)."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmr1l.so")

MR1L_OK = 0
MR1L_WARN_UNCOVERED = 16
C64, C128 = 0, 1
W_PAPER, W_EVAL = 0, 1
NSTAGES = 8

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_OVERFLOW", 3: "ERR_NOMEM", 4: "ERR_HIP", 5: "ERR_CALLBACK",
          6: "ERR_UNSUPPORTED", 16: "WARN_UNCOVERED"}

EXPORTED = ["mr1l_plan", "mr1l_plan_batched", "mr1l_forward", "mr1l_adjoint", "mr1l_alias", "mr1l_info", "mr1l_destroy",
            "mr1l_timing_enable", "mr1l_timing_read", "mr1l_cache_alias", "mr1l_memory_cache", "mr1l_fft_split", "mr1l_fft_p2_variant", "mr1l_work_limit", "mr1l_batch_inblock", "mr1l_rhs_interleave", "mr1l_fft_smooth", "mr1l_lsq_residual", "mr1l_lsq_residual_noalloc", "mr1l_construct", "sfft_detect",
            "sfft_sample_bspline", "sfft_bspline_coeffs", "sfft_bspline_l2_error", "mr1l_last_error", "mr1l_version"]


class Mr1lError(RuntimeError):
    def __init__(self, status: int, what: str, msg: str):
        super().__init__(f"{what}: {STATUS.get(status, status)}: {msg}")
        self.status = status


SAMPLER_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p)


class SfftPlanted(C.Structure):
    _fields_ = [("s", C.c_int64), ("freqs", C.c_void_p), ("coeffs", C.c_void_p), ("sigma", C.c_double),
                ("noise_seed", C.c_uint64)]


class SfftParams(C.Structure):
    _fields_ = [("delta", C.c_double), ("s", C.c_int64), ("s_local", C.c_int64), ("r", C.c_int),
                ("b", C.c_int), ("seed", C.c_uint64), ("dtype", C.c_int), ("c", C.c_double),
                ("gamma", C.c_double), ("zero_anchors", C.c_int), ("plain", C.c_int), ("redraw", C.c_int),
                ("order", C.c_void_p), ("delta_1d", C.c_double)]


SFFT_BSPLINE_MAX_TERMS = 8
SFFT_BSPLINE_MAX_ORDER = 12


class SfftBspline(C.Structure):
    _fields_ = [("terms", C.c_int), ("d", C.c_int), ("orders", C.c_void_p), ("weights", C.c_void_p),
                ("dtype", C.c_int)]


SFFT_MAX_D = 64


class SfftStats(C.Structure):
    _fields_ = [("d", C.c_int), ("n_It", C.c_int64 * SFFT_MAX_D), ("n_J", C.c_int64 * SFFT_MAX_D),
                ("n_detected", C.c_int64 * SFFT_MAX_D), ("L", C.c_int32 * SFFT_MAX_D),
                ("sumM", C.c_int64 * SFFT_MAX_D), ("calls", C.c_int32 * SFFT_MAX_D),
                ("redraws", C.c_int32 * SFFT_MAX_D),
                ("uncovered", C.c_int64 * SFFT_MAX_D), ("samples", C.c_int64),
                ("samples_full", C.c_int64), ("ms_sampling", C.c_double), ("ms_transform", C.c_double),
                ("ms_construct", C.c_double), ("ms_select", C.c_double), ("ms_total", C.c_double)]


_LIB = None


def lib() -> C.CDLL:
    """Load the library (raises if it has not been built: there is no fallback path)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    i32, i64, u64, vp, dbl = C.c_int, C.c_int64, C.c_uint64, C.c_void_p, C.c_double
    sig = {
        "mr1l_plan": [i32, i64, vp, i32, vp, vp, i32, i32, i64, i32, C.POINTER(vp)],
        "mr1l_plan_batched": [i32, i32, vp, vp, vp, vp, vp, i32, i32, i64, i32, C.POINTER(vp)],
        "mr1l_forward": [vp, vp, vp, vp],
        "mr1l_adjoint": [vp, vp, vp, vp],
        "mr1l_alias": [vp, vp, vp, vp, vp],
        "mr1l_info": [vp, vp, vp, vp],
        "mr1l_destroy": [vp],
        "mr1l_timing_enable": [vp, i32],
        "mr1l_cache_alias": [vp, i32],
        "mr1l_memory_cache": [i32, i64, C.POINTER(i64)],
        "mr1l_fft_split": [i32, i32, i32, C.POINTER(i32)],
        "mr1l_fft_p2_variant": [i32, i32, i32, C.POINTER(i32)],
        "mr1l_work_limit": [i64, C.POINTER(i64)],
        "mr1l_batch_inblock": [i32, C.POINTER(i32)],
        "mr1l_rhs_interleave": [i32, C.POINTER(i32)],
        "mr1l_fft_smooth": [i32, C.POINTER(i32)],
        "mr1l_lsq_residual": [vp, vp, vp, vp, vp, vp, vp],
        "mr1l_lsq_residual_noalloc": [vp, vp, vp, vp, vp, vp, vp],
        "mr1l_timing_read": [vp, vp, vp, vp],
        "mr1l_construct": [i32, i64, vp, dbl, dbl, i32, i32, u64, i64, i32, C.POINTER(i32), vp, vp,
                           C.POINTER(i32), C.POINTER(i64), i32],
        "sfft_detect": [i32, vp, vp, SAMPLER_FN, vp, C.POINTER(SfftPlanted), C.POINTER(SfftParams), i64,
                        C.POINTER(i64), vp, vp, C.POINTER(SfftStats), i32],
        "sfft_sample_bspline": [vp, i32, i64, vp, vp, vp],
        "sfft_bspline_coeffs": [C.POINTER(SfftBspline), i64, vp, vp],
        "sfft_bspline_l2_error": [C.POINTER(SfftBspline), i64, vp, vp, C.POINTER(dbl), C.POINTER(dbl)],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = C.c_int
    L.mr1l_last_error.restype = C.c_char_p
    L.mr1l_last_error.argtypes = []
    L.mr1l_version.restype = C.c_char_p
    L.mr1l_version.argtypes = []
    _LIB = L
    return L


def check(status: int, what: str, allow_warn: bool = True) -> int:
    if status == MR1L_OK or (allow_warn and status == MR1L_WARN_UNCOVERED):
        return status
    raise Mr1lError(status, what, lib().mr1l_last_error().decode(errors="replace"))
