"""ctypes declarations of libgivscore's C ABI (include/givscore.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgivscore.so")

GS_OK = 0
GS_EINVAL = -1
GS_ERANK = -2
GS_ENOMEM = -3
GS_EHIP = -4
GS_ENOTFINITE = -5
GS_ERANGE = -6
GS_OUT_BIC = 0
GS_OUT_RSS = 1
GS_MAX_M = 30

STATUS_NAMES = {
    GS_OK: "GS_OK", GS_EINVAL: "GS_EINVAL", GS_ERANK: "GS_ERANK", GS_ENOMEM: "GS_ENOMEM",
    GS_EHIP: "GS_EHIP", GS_ENOTFINITE: "GS_ENOTFINITE", GS_ERANGE: "GS_ERANGE",
}


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int), ("k", ctypes.c_int), ("ks", ctypes.c_int), ("q", ctypes.c_int),
        ("num_segments", ctypes.c_int64), ("sub_per_segment", ctypes.c_int64),
        ("swaps_per_segment", ctypes.c_int64), ("num_families", ctypes.c_int64),
        ("num_waves", ctypes.c_int64),
    ]


class ReduceOut(ctypes.Structure):
    _fields_ = [("best_score", ctypes.c_void_p), ("best_parents", ctypes.c_void_p),
                ("logsumexp", ctypes.c_void_p), ("top_score", ctypes.c_void_p),
                ("top_parents", ctypes.c_void_p), ("top_k", ctypes.c_int)]


class BatchData(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("ldx", ctypes.c_int64), ("scores", ctypes.c_void_p)]


class GivScoreError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libgivscore.so from the package directory.  There is no fallback: the
    library must have been built (``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc, gfx950) before using the package")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, u64, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
    pplan = ctypes.POINTER(vp)
    sig = {
        "gs_num_families": (i64, [i32]),
        "gs_family_index": (i64, [i32, i32, u64]),
        "gs_upsilon": (i64, [i32, ctypes.POINTER(ctypes.c_int32), i64]),
        "gs_plan": (i32, [i32, pplan]),
        "gs_plan_tuned": (i32, [i32, i32, i32, pplan]),
        "gs_plan_destroy": (None, [vp]),
        "gs_plan_get_info": (i32, [vp, ctypes.POINTER(PlanInfo)]),
        "gs_plan_workspace_bytes": (i32, [vp, i64, i32, ctypes.POINTER(i64)]),
        "gs_plan_count_emissions": (i32, [vp, ctypes.POINTER(ctypes.c_int32), i64]),
        "gs_qr_r0": (i32, [vp, vp, i64, i32, i64, vp, vp]),
        "gs_score_all": (i32, [vp, vp, i64, i32, i64, vp, i32, vp]),
        "gs_score_all_f64": (i32, [vp, vp, i64, i32, i64, vp, i32, vp]),
        "gs_count_writes": (i32, [vp, vp, i64, i32, i64, vp, vp]),
        "gs_score_beta": (i32, [vp, vp, i64, i32, i64, vp, vp]),
        "gs_score_reduce": (i32, [vp, vp, i64, i32, i64, ctypes.POINTER(ReduceOut), vp]),
        "gs_score_all_static": (i32, [vp, vp, i64, i32, i64, vp, i32, vp, vp]),
        "gs_score_all_many": (i32, [vp, i32, ctypes.POINTER(vp), i64, i64, ctypes.POINTER(vp),
                                    i32, i32, vp]),
        "gs_many_status": (i32, [vp, ctypes.POINTER(ctypes.c_int)]),
        "gs_score_backward": (i32, [vp, vp, i64, i32, i64, vp, i32, vp, i64, vp]),
        "gs_score_backward_f64": (i32, [vp, vp, i64, i32, i64, vp, i32, vp, i64, vp]),
        "gs_plan_set_reuse": (i32, [vp, i32]),
        "gs_sync_status": (i32, [vp]),
        "gs_column_vif": (i32, [vp, ctypes.POINTER(ctypes.c_double)]),
        "gs_set_timing": (i32, [vp, i32]),
        "gs_get_timing": (i32, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]),
        "gs_batch_create": (i32, [i32, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(i64),
                                  ctypes.POINTER(ctypes.c_int), pplan]),
        "gs_batch_destroy": (None, [vp]),
        "gs_batch_info": (i32, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                ctypes.POINTER(i64)]),
        "gs_score_batched": (i32, [vp, ctypes.POINTER(BatchData), i32, i32, vp]),
        "gs_batch_status": (i32, [vp, ctypes.POINTER(ctypes.c_int)]),
        "gs_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    msg = lib().gs_last_error()
    return msg.decode() if msg else ""


def check(code: int) -> int:
    if code < 0:
        raise GivScoreError(code, last_error())
    return code
