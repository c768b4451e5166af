"""ctypes declarations of the libhomog C ABI (include/homog.h).

Loading is lazy; ``lib()`` raises if the shared library has not been built.
There is no fallback implementation: every computation runs in libhomog.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhomog.so")

HG_OK, HG_EINVAL, HG_EHIP, HG_EWORKSPACE, HG_EUNSUPPORTED = 0, -1, -2, -3, -4
HG_ACA, HG_SKS = 0, 1

vp = C.c_void_p
i32 = C.c_int32
i64 = C.c_int64
u64 = C.c_uint64
f32 = C.c_float
sz = C.c_size_t


class Tuning(C.Structure):
    _fields_ = [("pts_per_lane", i32), ("hyps_per_block", i32), ("blocks_per_cu", i32),
                ("reserved", i32)]


# name -> (restype, argtypes); the order of argtypes follows homog.h
SIGNATURES = {
    "hg_status_str": (C.c_char_p, [C.c_int]),
    "hg_last_error": (C.c_char_p, []),
    "hg_version": (C.c_int, []),
    "hg_solve4": (C.c_int, [C.c_int, vp, vp, i64, i64, vp, vp, vp]),
    "hg_stream_copy": (C.c_int, [vp, vp, i64, vp]),
    "hg_stream_planes": (C.c_int, [vp, i32, vp, i32, vp, i64, i64, vp]),
    "hg_solve_sk": (C.c_int, [C.POINTER(C.c_double), vp, i64, i64, vp, vp,
                              C.POINTER(C.c_double), vp]),
    "hg_solve3_affine": (C.c_int, [vp, vp, i64, i64, vp, vp, vp]),
    "hg_ransac_ws_bytes": (sz, [i32, i32]),
    "hg_ransac": (C.c_int, [vp, i32, i64, i32, f32, u64, vp, vp, vp, vp, vp, vp, sz, vp]),
    "hg_ransac_plain": (C.c_int, [vp, i32, i64, i32, f32, u64, vp, vp, vp, vp, vp, vp, sz, vp]),
    "hg_ransac_noalloc": (C.c_int, [vp, i32, i64, i32, f32, u64, vp, vp, vp, vp, vp, vp]),
    "hg_ransac_batched_ws_bytes": (sz, [i32, i32]),
    "hg_ransac_batched": (C.c_int, [vp, i64, vp, i32, i32, f32, u64, C.POINTER(Tuning),
                                    vp, vp, vp, vp, vp, vp, sz, vp]),
    "hg_ransac_adaptive_ws_bytes": (sz, [i32, i32]),
    "hg_ransac_adaptive": (C.c_int, [vp, i64, vp, i32, i32, f32, u64, C.c_double,
                                     C.POINTER(Tuning), vp, vp, vp, vp, vp, vp, sz, vp]),
    "hg_ransac_autotune": (C.c_int, [vp, i64, vp, vp, i32, i32, f32, u64, vp, sz, vp,
                                     C.POINTER(Tuning)]),
    "hg_ransac_batched_graph_create": (C.c_int, [vp, i64, vp, i32, i32, f32, u64,
                                                 C.POINTER(Tuning), vp, vp, vp, vp, vp, vp, sz,
                                                 vp, C.POINTER(vp)]),
    "hg_refit_ho": (C.c_int, [vp, i64, vp, i32, vp, vp, vp, vp, vp]),
    "hg_graph_launch": (C.c_int, [vp, vp]),
    "hg_graph_destroy": (None, [vp]),
    "hg_aca_rect_fwd": (C.c_int, [vp, i32, f32, f32, f32, f32, vp, vp]),
    "hg_aca_rect_bwd": (C.c_int, [vp, vp, i32, f32, f32, f32, f32, vp, vp]),
    "hg_aca_fwd": (C.c_int, [vp, vp, i32, vp, vp]),
    "hg_aca_bwd": (C.c_int, [vp, vp, vp, i32, vp, vp, vp]),
    "hg_photometric_fwd": (C.c_int, [vp, vp, vp, i32, i32, i32, vp, vp]),
    "hg_photometric_bwd": (C.c_int, [vp, vp, vp, vp, i32, i32, i32, vp, vp]),
    "hg_photometric_fwd_grad": (C.c_int, [vp, vp, vp, i32, i32, i32, vp, vp, vp]),
    "hg_scale_grad": (C.c_int, [vp, vp, i32, vp, vp]),
    "hg_refine": (C.c_int, [vp, vp, i32, i32, i32, i32, f32, vp, vp, vp]),
    "hg_refine_graph_create": (C.c_int, [vp, vp, i32, i32, i32, i32, f32, vp, vp, vp,
                                         C.POINTER(vp)]),
    "hg_warp_l1_fwd": (C.c_int, [vp, vp, vp, i32, i32, i32, vp, vp]),
    "hg_warp_l1_bwd": (C.c_int, [vp, vp, vp, vp, i32, i32, i32, vp, vp]),
    "hg_warp_store_fwd": (C.c_int, [vp, vp, i32, i32, i32, vp, vp]),
    "hg_l1_fwd": (C.c_int, [vp, vp, i32, i32, i32, vp, vp]),
    "hg_l1_bwd": (C.c_int, [vp, vp, vp, i32, i32, i32, vp, vp]),
    "hg_warp_bwd_from_grad": (C.c_int, [vp, vp, vp, i32, i32, i32, vp, vp]),
}

_lib = None
_lock = threading.Lock()


class HomogError(RuntimeError):
    def __init__(self, fn, status, detail):
        super().__init__(f"{fn} returned {status}: {detail}")
        self.status = status


def lib():
    """The loaded libhomog (declared signatures); raises if it is not built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: build it with `python -m paper_2402_18008_amd.build`")
            L = C.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                if not hasattr(L, name):
                    continue
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def check(fn_name, status):
    if status != HG_OK:
        detail = lib().hg_last_error().decode(errors="replace")
        raise HomogError(fn_name, status, detail)
    return status


def call(name, *args):
    """Call a status-returning entry point and raise HomogError on failure."""
    return check(name, getattr(lib(), name)(*args))
