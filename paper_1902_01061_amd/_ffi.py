"""ctypes declarations of the C ABI in include/sgreg.h (marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgreg.so")

SGR_OK = 0
SGR_EINVAL = -1
SGR_EDEGENERATE = -2
SGR_EHIP = -3
SGR_ENOMEM = -4
SGR_ENUMERIC = -5


class SgrCloud(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("m", ctypes.c_void_p), ("n", ctypes.c_int64)]


class SgrParams(ctypes.Structure):
    _fields_ = [("p", ctypes.c_double), ("g_mode", ctypes.c_int32), ("k", ctypes.c_int32),
                ("sigma", ctypes.c_double), ("eps", ctypes.c_double), ("G1", ctypes.c_double),
                ("E", ctypes.c_int32), ("flags", ctypes.c_int32), ("dt2", ctypes.c_double),
                ("momentum", ctypes.c_double)]


class SgrLevel(ctypes.Structure):
    _fields_ = [("radius_scale", ctypes.c_double), ("sigma_scale", ctypes.c_double), ("iters", ctypes.c_int32),
                ("k", ctypes.c_int32)]


class SgrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sgreg error {code}: {msg}")
        self.code = code


_lib = None

P = ctypes.c_void_p
I = ctypes.c_int
I64 = ctypes.c_int64
D = ctypes.c_double
CP = ctypes.POINTER(SgrCloud)
PP = ctypes.POINTER(SgrParams)

SIGNATURES = {
    "sgr_create": [ctypes.POINTER(P), I],
    "sgr_destroy": [P],
    "sgr_descriptors": [P, CP, I, P, P, P],
    "sgr_knn": [P, CP, I, P, P],
    "sgr_descriptors_batch": [P, I, CP, I, P, P, P],
    "sgr_step": [P, CP, P, CP, P, P, P, PP, I, P, P, P, P, P],
    "sgr_step_static": [P, CP, P, CP, P, P, P, PP, I, P, P, P, P, P],
    "sgr_register": [P, CP, CP, PP, P, P, P],
    "sgr_residual": [P, CP, CP, P, P, P, P],
    "sgr_plan_create": [P, CP, P, CP, P, P, P, PP, ctypes.POINTER(P), P],
    "sgr_plan_destroy": [P],
    "sgr_plan_force": [P, I, D, P, P, P, P],
    "sgr_plan_step": [P, I, P, P, P, P],
    "sgr_set_tiles": [P, I64, I64, D, I, I, I],
    "sgr_force_fwd": [P, CP, P, CP, P, P, PP, D, P, P, P],
    "sgr_register_batch": [P, I, CP, CP, PP, P, P, P, P],
    "sgr_autotune": [P, CP, P, CP, P, P, P, PP, I, P, P, P],
    "sgr_tiles_save": [P, ctypes.c_char_p],
    "sgr_tiles_load": [P, ctypes.c_char_p],
    "sgr_multistart": [P, CP, CP, PP, I, P, P, P, P, P],
    "sgr_force_bwd": [P, CP, P, CP, P, P, PP, D, P, P, P, P, P, P, P],
    "sgr_unrolled_fwd": [P, CP, P, CP, P, P, P, PP, I, P, P, P],
    "sgr_unrolled_bwd": [P, CP, P, CP, P, P, P, PP, I, P, P, P, P, P],
    "sgr_change_detect": [P, CP, P, CP, P, P, D, D, D, P, P, P, P],
    "sgr_descriptors_radius": [P, CP, ctypes.c_float, P, P, P],
    "sgr_register_pyramid": [P, CP, CP, PP, ctypes.POINTER(SgrLevel), I, P, P, P],
    "sgr_descriptors_hn": [P, CP, I, I, P, P],
    "sgr_descriptors_poly": [P, CP, I, P, P],
    "sgr_step_vec": [P, CP, P, CP, P, I, P, P, PP, I, P, P, P, P, P],
    "sgr_register_vec": [P, CP, P, CP, P, I, PP, P, P, P],
}


def lib():
    """Load libsgreg.so.  There is no fallback: without the built library
    every call fails loudly."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1902_01061_amd.build` "
                              "(hipcc, gfx950); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.sgr_last_error.argtypes = []
        L.sgr_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(code: int):
    if code != SGR_OK:
        raise SgrError(code, lib().sgr_last_error().decode(errors="replace"))
