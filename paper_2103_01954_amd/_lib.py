"""ctypes binding of libmvp.so (include/mvp.h): argument marshalling only.

Each C entry point is exposed under its own name with its C signature.  The
library must have been built (``python -m paper_2103_01954_amd.build``); there is
no fallback implementation, so a missing library raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmvp.so")

MVP_OK, MVP_ERR_INVALID, MVP_ERR_OOM, MVP_ERR_DEVICE, MVP_ERR_BUSY, MVP_ERR_NOT_READY = range(6)
MVP_F32, MVP_BF16 = 0, 1
STATUS_NAMES = {0: "MVP_OK", 1: "MVP_ERR_INVALID", 2: "MVP_ERR_OOM", 3: "MVP_ERR_DEVICE",
                4: "MVP_ERR_BUSY", 5: "MVP_ERR_NOT_READY"}


class mvp_prims(C.Structure):
    _fields_ = [("n_prim", C.c_int32), ("M", C.c_int32), ("payload_dtype", C.c_int32),
                ("reserved", C.c_int32), ("pos", C.c_void_p), ("rot", C.c_void_p),
                ("scale", C.c_void_p), ("payload", C.c_void_p)]


MVP_COMBINE_SUM, MVP_COMBINE_SEQUENTIAL = 0, 1
MVP_KERNEL_FWD_MARCH, MVP_KERNEL_BWD_MARCH = 0, 1
MVP_NOALLOC_MAX_RAYS = 1048576


class mvp_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("origin", C.c_float * 3),
                ("pix2dir", C.c_float * 9)]


class mvp_march_params(C.Structure):
    _fields_ = [("step", C.c_float), ("eps_early", C.c_float), ("t_near", C.c_float),
                ("fade_alpha", C.c_float), ("fade_beta", C.c_float), ("combine", C.c_int32)]


class mvp_ray_aux(C.Structure):
    _fields_ = [("j_end", C.c_int32), ("t_prev", C.c_float)]


class mvp_accel_info(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("n_prim", C.c_int32), ("n_tile_pairs", C.c_int64), ("n_ray_pairs", C.c_int64),
                ("device_bytes", C.c_int64), ("pairs_in_forward", C.c_int32), ("reserved", C.c_int32)]


class mvp_request(C.Structure):
    _fields_ = [("scene_id", C.c_uint64), ("cam", mvp_camera), ("params", mvp_march_params),
                ("rgba_out", C.c_void_p)]


P = C.c_void_p
PP = C.POINTER(C.c_void_p)
_SIGS = {
    "mvp_create": ([C.c_int, PP], C.c_int),
    "mvp_destroy": ([P], C.c_int),
    "mvp_last_error": ([], C.c_char_p),
    "mvp_version": ([], C.c_char_p),
    "mvp_build_accel": ([P, C.POINTER(mvp_prims), C.POINTER(mvp_camera), C.c_int32,
                         C.POINTER(mvp_march_params), PP, P], C.c_int),
    "mvp_build_accel_rays": ([P, C.POINTER(mvp_prims), C.POINTER(mvp_camera), C.c_int32,
                              C.POINTER(mvp_march_params), P, C.c_int64, PP, P], C.c_int),
    "mvp_accel_destroy": ([P, P, P], C.c_int),
    "mvp_accel_get_info": ([P, C.POINTER(mvp_accel_info)], C.c_int),
    "mvp_render_fwd": ([P, P, C.POINTER(mvp_prims), P, P, P], C.c_int),
    "mvp_render_bwd": ([P, P, C.POINTER(mvp_prims), P, P, P, P, P, P, P], C.c_int),
    "mvp_render_bwd_noalloc": ([P, P, C.POINTER(mvp_prims), P, P, P, P, P, P, P], C.c_int),
    "mvp_render_fwd_bg": ([P, P, C.POINTER(mvp_prims), P, P, P, P], C.c_int),
    "mvp_render_bwd_bg": ([P, P, C.POINTER(mvp_prims), P, P, P, P, P, P, P, P, P, P], C.c_int),
    "mvp_accel_counts": ([P, P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), P], C.c_int),
    "mvp_accel_load_counts": ([P, P, C.POINTER(C.c_uint64), P], C.c_int),
    "mvp_debug_hits": ([P, P, C.POINTER(mvp_prims), P, P, C.c_int64, C.POINTER(C.c_int64), P], C.c_int),
    "mvp_timing_start": ([P, C.c_int32], C.c_int),
    "mvp_timing_read": ([P, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_int32)], C.c_int),
    "mvp_timing_stop": ([P], C.c_int),
    "mvp_serve_configure": ([P, C.c_size_t, C.c_int32], C.c_int),
    "mvp_scene_create": ([P, C.POINTER(mvp_prims), C.POINTER(C.c_uint64)], C.c_int),
    "mvp_scene_release": ([P, C.c_uint64], C.c_int),
    "mvp_submit": ([P, C.POINTER(mvp_request), C.POINTER(C.c_uint64)], C.c_int),
    "mvp_poll": ([P, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "mvp_ticket_times": ([P, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_double),
                          C.POINTER(C.c_double)], C.c_int),
    "mvp_clock": ([], C.c_double),
    "mvp_wait": ([P, C.c_uint64, C.c_double], C.c_int),
    "mvp_ticket_release": ([P, C.c_uint64], C.c_int),
    "mvp_ticket_samples": ([P, C.c_uint64, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)], C.c_int),
}
EXPORTS = tuple(_SIGS)

_lib = None


def load(path: str = LIB_PATH):
    """Load libmvp.so once and attach the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2103_01954_amd.build`")
    lib = C.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name, None)
        if fn is None:      # an older build; the export test checks the full set
            continue
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class MVPError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} returned {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(fn: str, status: int):
    if status != MVP_OK:
        raise MVPError(fn, status, load().mvp_last_error().decode(errors="replace"))


def __getattr__(name):
    if name in _SIGS:
        return getattr(load(), name)
    raise AttributeError(name)
