"""ctypes binding of libboys.so (argument marshalling only; see include/boys.h).

The library is loaded from this package directory.  If it is missing, every entry point
raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libboys.so")

FP64 = 0
FP32 = 1
FP64_PLUS = 2
FP32X = 3
FP32S = 4

OK = 0
ERR_INVALID_ARGUMENT = 1
ERR_UNSUPPORTED_NMAX = 2
ERR_OUT_OF_MEMORY = 3
ERR_DEVICE = 4
ERR_TOO_LARGE = 5

# every function declared in include/boys.h
EXPORTS = (
    "boys_eval",
    "boys_eval_rows",
    "boys_eval_split",
    "boys_eri_ssss",
    "boys_eval_batched",
    "boys_eval_batched_noalloc",
    "boys_plan_create",
    "boys_plan_update",
    "boys_plan_execute",
    "boys_plan_destroy",
    "boys_autotune",
    "boys_server_create",
    "boys_server_submit",
    "boys_server_poll",
    "boys_server_result",
    "boys_server_copy_result",
    "boys_server_release",
    "boys_server_get_stats",
    "boys_server_drain",
    "boys_server_destroy",
    "boys_max_nmax",
    "boys_cutoff",
    "boys_status_string",
)


class BoysArray(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("out", ctypes.c_void_p), ("n", ctypes.c_int64),
                ("ld_out", ctypes.c_int64), ("n_max", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


class BoysTuning(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("block", ctypes.c_int32),
                ("grid_per_cu", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("order", ctypes.c_int32), ("split_nmax", ctypes.c_int32)]


class BoysServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("streams", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("max_tiles", ctypes.c_int32)]


class BoysPairList(ctypes.Structure):
    _fields_ = [("p", ctypes.c_void_p), ("px", ctypes.c_void_p), ("py", ctypes.c_void_p),
                ("pz", ctypes.c_void_p), ("w", ctypes.c_void_p), ("start", ctypes.c_void_p),
                ("count", ctypes.c_int32)]


class BoysServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in (
        "submitted", "admitted", "launched", "completed", "released", "batches",
        "queued_now", "inflight_now", "max_queued", "max_inflight",
        "bytes_in_use", "max_bytes_in_use", "device_errors", "failed")]


class BoysError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} (status {status})")


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2504_07637_amd.build` "
                "(there is no non-HIP fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.boys_eval.argtypes = [vp, i64, i32, vp, i64, i32, vp]
        L.boys_eval.restype = ctypes.c_int
        L.boys_eval_rows.argtypes = [vp, i64, i32, ctypes.c_uint64, vp, i64, i32, vp]
        L.boys_eval_rows.restype = ctypes.c_int
        L.boys_eval_split.argtypes = [vp, i64, i32, i32, vp, i64, vp]
        L.boys_eval_split.restype = ctypes.c_int
        L.boys_eri_ssss.argtypes = [ctypes.POINTER(BoysPairList), ctypes.POINTER(BoysPairList),
                                    i32, vp, i64, vp]
        L.boys_eri_ssss.restype = ctypes.c_int
        L.boys_eval_batched.argtypes = [ctypes.POINTER(BoysArray), i32, vp]
        L.boys_eval_batched.restype = ctypes.c_int
        L.boys_eval_batched_noalloc.argtypes = [ctypes.POINTER(BoysArray), i32, vp]
        L.boys_eval_batched_noalloc.restype = ctypes.c_int
        L.boys_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(BoysArray), i32,
                                       ctypes.POINTER(BoysTuning)]
        L.boys_plan_create.restype = ctypes.c_int
        L.boys_plan_update.argtypes = [vp, ctypes.POINTER(BoysArray), i32]
        L.boys_plan_update.restype = ctypes.c_int
        L.boys_plan_execute.argtypes = [vp, vp]
        L.boys_plan_execute.restype = ctypes.c_int
        L.boys_plan_destroy.argtypes = [vp]
        L.boys_plan_destroy.restype = None
        L.boys_autotune.argtypes = [ctypes.POINTER(BoysArray), i32, ctypes.POINTER(BoysTuning),
                                    i32, i32, i32, vp, ctypes.POINTER(BoysTuning),
                                    ctypes.POINTER(ctypes.c_float)]
        L.boys_autotune.restype = ctypes.c_int
        u64p = ctypes.POINTER(ctypes.c_uint64)
        dpp = ctypes.POINTER(ctypes.c_double)
        L.boys_server_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(BoysServerConfig)]
        L.boys_server_submit.argtypes = [vp, vp, i64, i32, i32, u64p]
        L.boys_server_poll.argtypes = [vp, u64p, i32]
        L.boys_server_poll.restype = i32
        L.boys_server_result.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(vp),
                                         ctypes.POINTER(i64), dpp, dpp]
        L.boys_server_copy_result.argtypes = [vp, ctypes.c_uint64, vp, i64, vp]
        L.boys_server_release.argtypes = [vp, ctypes.c_uint64]
        L.boys_server_get_stats.argtypes = [vp, ctypes.POINTER(BoysServerStats)]
        L.boys_server_drain.argtypes = [vp, ctypes.c_double]
        L.boys_server_destroy.argtypes = [vp]
        L.boys_server_destroy.restype = None
        for f in (L.boys_server_create, L.boys_server_submit, L.boys_server_result,
                  L.boys_server_copy_result, L.boys_server_release, L.boys_server_get_stats,
                  L.boys_server_drain):
            f.restype = ctypes.c_int
        L.boys_max_nmax.argtypes = [i32]
        L.boys_max_nmax.restype = i32
        L.boys_cutoff.argtypes = [i32, i32]
        L.boys_cutoff.restype = ctypes.c_double
        L.boys_status_string.argtypes = [ctypes.c_int]
        L.boys_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().boys_status_string(status).decode()


def check(status: int, where: str) -> None:
    if status != OK:
        raise BoysError(status, where)
