"""ctypes declarations of libwsconv.so (the C-ABI in include/wsconv.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwsconv.so")

WS_OK = 0
WS_EINVAL = -1
WS_EUNSUPPORTED = -2
WS_EDEVICE = -3

WS_LOG, WS_POWER, WS_HELMHOLTZ, WS_YUKAWA = 0, 1, 2, 3
WS_FP64, WS_FP32 = 0, 1
WS_FS_NONE, WS_FS_DISC, WS_FS_SQUARE = 0, 1, 2
WS_LS_CONVERGED, WS_LS_MAXIT, WS_LS_BREAKDOWN = 0, 1, 2


class WsKernel(ctypes.Structure):
    _fields_ = [("family", c_int), ("scale", c_double), ("gamma", c_double), ("kappa", c_double),
                ("beta", c_double)]


class WsGrid(ctypes.Structure):
    _fields_ = [("n", c_int), ("b", c_int), ("a", c_double), ("support_radius", c_double), ("force_a", c_int)]


class WsFsDesc(ctypes.Structure):
    _fields_ = [("shape", c_int), ("c1", c_double), ("c2", c_double), ("size", c_double),
                ("psi_r1", c_double), ("psi_r2", c_double)]


class WsLsInfo(ctypes.Structure):
    _fields_ = [("status", c_int), ("iterations", c_int), ("matvecs", c_int),
                ("refinements", c_int), ("rel_residual", c_double)]


WS_REQ_APPLY, WS_REQ_LS = 0, 1


class WsServeConfig(ctypes.Structure):
    _fields_ = [("precision", c_int), ("streams", c_int), ("max_batch", c_int), ("max_plans", c_int),
                ("max_skips", c_int), ("mix_plans", c_int)]


class WsRequest(ctypes.Structure):
    _fields_ = [("kind", c_int), ("kernel", WsKernel), ("n", c_int), ("input", c_void_p),
                ("contrast", c_void_p), ("output", c_void_p), ("tol", c_double), ("restart", c_int),
                ("max_matvecs", c_int)]


class WsResult(ctypes.Structure):
    _fields_ = [("status", c_int), ("batch", c_int), ("t_submit", c_double), ("t_start", c_double),
                ("t_done", c_double), ("ls", WsLsInfo)]


class WsServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_ulonglong), ("completed", ctypes.c_ulonglong),
                ("launches", ctypes.c_ulonglong), ("plan_builds", ctypes.c_ulonglong),
                ("plan_evictions", ctypes.c_ulonglong), ("arena_bytes", c_size_t),
                ("arena_peak_bytes", c_size_t), ("cached_plans", c_int), ("pending", c_int)]


EXPORTS = {
    "conv_plan_query": (c_int, [POINTER(WsKernel), POINTER(WsGrid), c_int, POINTER(c_size_t), POINTER(c_size_t)]),
    "conv_plan": (c_int, [POINTER(WsKernel), POINTER(WsGrid), c_int, c_void_p, c_void_p, POINTER(c_void_p)]),
    "conv_plan_radius": (c_double, [c_void_p]),
    "conv_apply": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, POINTER(WsFsDesc), c_void_p]),
    "conv_apply_chunk": (c_int, [c_void_p]),
    "conv_apply_noalloc": (c_int, [c_void_p, c_int, c_void_p, c_void_p, POINTER(WsFsDesc), c_void_p]),
    "conv_apply_multi": (c_int, [c_int, POINTER(c_void_p), POINTER(c_int), POINTER(c_void_p), POINTER(c_void_p),
                                 POINTER(c_void_p), c_void_p]),
    "conv_apply_pass": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ls_solve_query": (c_int, [c_void_p, c_int, c_int, POINTER(c_size_t)]),
    "ls_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int, c_int, c_int, c_void_p, c_void_p,
                         POINTER(WsLsInfo), c_void_p]),
    "ls_solve_batch_query": (c_int, [c_void_p, c_int, c_int, c_int, POINTER(c_size_t)]),
    "ls_solve_batch": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_double, c_int, c_int, c_int, c_void_p,
                               c_void_p, POINTER(WsLsInfo), c_void_p]),
    "conv_eval_query": (c_int, [c_void_p, POINTER(c_size_t)]),
    "conv_eval": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ls_solve_fs_query": (c_int, [c_void_p, POINTER(WsFsDesc), c_int, c_int, POINTER(c_size_t)]),
    "ls_solve_fs": (c_int, [c_void_p, c_void_p, POINTER(WsFsDesc), c_void_p, c_double, c_int, c_int, c_int,
                            c_void_p, c_void_p, POINTER(WsLsInfo), c_void_p]),
    "conv_plan_moments": (c_int, [c_void_p, c_int, POINTER(c_int), POINTER(c_int), POINTER(c_double), c_void_p]),
    "conv_destroy": (None, [c_void_p]),
    "serve_footprint": (c_int, [POINTER(WsServeConfig), POINTER(WsRequest), POINTER(c_size_t)]),
    "serve_create": (c_int, [POINTER(WsServeConfig), c_void_p, c_size_t, POINTER(c_void_p)]),
    "serve_submit": (c_int, [c_void_p, POINTER(WsRequest), POINTER(ctypes.c_ulonglong)]),
    "serve_wait": (c_int, [c_void_p, ctypes.c_ulonglong, c_double, POINTER(WsResult)]),
    "serve_now": (c_double, [c_void_p]),
    "serve_stats": (c_int, [c_void_p, POINTER(WsServeStats)]),
    "serve_destroy": (None, [c_void_p]),
    "conv_last_error": (ctypes.c_char_p, []),
}

_lib = None


class WsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"wsconv error {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load libwsconv.so (raises if it is missing: the HIP library is the only implementation)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing; build it with `python -m paper_2107_03958_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> int:
    if rc < 0:
        msg = load().conv_last_error().decode(errors="replace")
        raise WsError(rc, msg)
    return rc
