"""ctypes binding of ``libftm.so`` (argument marshalling only).

torch is imported before the library is loaded so that the HIP runtime torch
already holds (soname ``libamdhip64.so.7``) is the one the library binds to:
device pointers and streams are then shared between the two.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime first, see above)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libftm.so")

# ftm_status
OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_OOM, ERR_BUDGET, ERR_HIP, ERR_STATE = range(7)
# ftm_dtype
F64, F32, F16, BF16 = range(4)
# ftm_rhs_mode
RHS_AUTO, RHS_GEMV, RHS_GEMM = range(3)
# ftm_tuning.fft_shape: default, fixed-plan large / small tile, runtime-plan
FFT_DEFAULT, FFT_FIXED, FFT_FIXED_SMALL, FFT_GENERIC = range(4)
# ftm_gemv_type, ftm_gemv_op
TYPE_S, TYPE_D, TYPE_C, TYPE_Z = range(4)
OP_N, OP_T, OP_C = range(3)
# FTM_SCRATCH_BYTES: size of the static scratch workspace of ftm_apply_scratch
SCRATCH_BYTES = 96 << 20

# Every symbol include/ftm.h declares.
EXPORTS = ("ftm_setup_operator", "ftm_setup_operator_strided", "ftm_set_precision", "ftm_matvec", "ftm_rmatvec",
           "ftm_workspace_size", "ftm_apply", "ftm_apply_scratch",
           "ftm_hessian_workspace_size", "ftm_hessian_apply", "ftm_round", "ftm_select_precision",
           "ftm_get_spectrum", "ftm_operator_info", "ftm_profile_enable", "ftm_profile_read",
           "ftm_set_rhs_mode", "ftm_set_gemm_crossover", "ftm_autotune", "ftm_get_tuning",
           "ftm_set_tuning", "ftm_graph_create", "ftm_graph_launch", "ftm_graph_destroy",
           "ftm_server_create", "ftm_server_submit", "ftm_server_poll", "ftm_server_wait",
           "ftm_server_latencies", "ftm_server_get_stats", "ftm_server_destroy",
           "ftm_destroy_operator", "ftm_sbgemv",
           "ftm_status_string", "ftm_last_error")


class FtmPrecision(ctypes.Structure):
    _fields_ = [("pad", ctypes.c_int32), ("fft", ctypes.c_int32), ("gemv", ctypes.c_int32),
                ("ifft", ctypes.c_int32), ("unpad", ctypes.c_int32), ("accum", ctypes.c_int32)]


class FtmTuning(ctypes.Structure):
    _fields_ = [("gemv_variant", ctypes.c_int32 * 2), ("fft_shape", (ctypes.c_int32 * 2) * 2),
                ("gemm_tile", ctypes.c_int32 * 2), ("gemm_kind", ctypes.c_int32 * 2),
                ("gemm_min_rhs", ctypes.c_int64 * 2),
                ("ms", ctypes.c_double * 2)]


class FtmServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("rhs_launched", ctypes.c_uint64),
                ("coalesced_requests", ctypes.c_uint64), ("budget_waits", ctypes.c_uint64),
                ("max_inflight_requests", ctypes.c_int64), ("queued_requests", ctypes.c_int64),
                ("peak_workspace_bytes", ctypes.c_size_t), ("workspace_in_use_bytes", ctypes.c_size_t)]


class FtmError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func} failed: status {status} ({msg})")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load the library once; fails loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(python paper_2508_10202_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
    prec_p = ctypes.POINTER(FtmPrecision)
    sigs = {
        "ftm_setup_operator": [ctypes.POINTER(vp), vp, i64, i64, i64, prec_p, prec_p, u32, i64, vp],
        "ftm_setup_operator_strided": [ctypes.POINTER(vp), vp, i64, i64, i64, i64, i64, i64, prec_p, prec_p, u32,
                                       i64, vp],
        "ftm_set_precision": [vp, prec_p, prec_p],
        "ftm_matvec": [vp, vp, vp, i64, vp],
        "ftm_rmatvec": [vp, vp, vp, i64, vp],
        "ftm_workspace_size": [vp, i32, i64, ctypes.POINTER(ctypes.c_size_t)],
        "ftm_apply": [vp, i32, vp, vp, i64, vp, ctypes.c_size_t, vp],
        "ftm_apply_scratch": [vp, i32, vp, vp, i64, vp],
        "ftm_hessian_workspace_size": [vp, i64, ctypes.POINTER(ctypes.c_size_t)],
        "ftm_hessian_apply": [vp, vp, vp, i64, vp, ctypes.c_size_t, vp],
        "ftm_round": [i32, i32, vp, vp, i64, vp],
        "ftm_select_precision": [vp, i32, ctypes.c_double, vp, i32, prec_p, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double), vp],
        "ftm_get_spectrum": [vp, i32, i64, i64, vp, vp],
        "ftm_operator_info": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                              ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_size_t)],
        "ftm_profile_enable": [vp, i32],
        "ftm_set_rhs_mode": [vp, i32],
        "ftm_set_gemm_crossover": [vp, i64],
        "ftm_autotune": [vp, i32, vp],
        "ftm_get_tuning": [vp, ctypes.POINTER(FtmTuning)],
        "ftm_set_tuning": [vp, ctypes.POINTER(FtmTuning)],
        "ftm_graph_create": [ctypes.POINTER(vp), vp, i32, vp, vp, i64],
        "ftm_graph_launch": [vp, vp],
        "ftm_graph_destroy": [vp],
        "ftm_profile_read": [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), i32],
        "ftm_destroy_operator": [vp],
        "ftm_server_create": [ctypes.POINTER(vp), ctypes.c_size_t, i32, i64],
        "ftm_server_submit": [vp, vp, i32, vp, vp, i64, vp, ctypes.POINTER(ctypes.c_uint64)],
        "ftm_server_poll": [vp, ctypes.c_uint64, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)],
        "ftm_server_wait": [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double), ctypes.c_double],
        "ftm_server_latencies": [vp, ctypes.c_uint64, i64, ctypes.POINTER(ctypes.c_double)],
        "ftm_server_get_stats": [vp, ctypes.POINTER(FtmServerStats)],
        "ftm_server_destroy": [vp],
        "ftm_sbgemv": [i32, i32, i64, i64, vp, vp, i64, i64, vp, i64, vp, vp, i64, i64, vp],
    }
    for name, args in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.ftm_status_string.argtypes = [ctypes.c_int]
    L.ftm_status_string.restype = ctypes.c_char_p
    L.ftm_last_error.argtypes = []
    L.ftm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status: int, func: str) -> None:
    if status != OK:
        L = lib()
        raise FtmError(status, func, (L.ftm_last_error() or b"").decode())
