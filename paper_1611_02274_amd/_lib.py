"""ctypes declarations of librkmi.so (include/rkmi.h).

The library is loaded from this package's directory.  There is no fallback: if
it is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librkmi.so")

RK_OK, RK_EINVAL, RK_ENOMEM, RK_EHIP, RK_EUNSUPPORTED, RK_EWORKSPACE = 0, -1, -2, -3, -4, -5
RK_SYS_OK, RK_SYS_NONFINITE, RK_SYS_HMIN, RK_SYS_MAXSTEPS = 0, 1, 2, 3
RK_NSTATS = 6
RK_METHOD_RKCK, RK_METHOD_RKC = 0, 1

EXPORTS = (
    "rk_version", "rk_last_error", "rk_problem_create_vdp", "rk_problem_create_mass_action",
    "rk_problem_destroy", "rk_problem_dims", "rk_workspace_bytes", "rk_integrate_rkck",
    "rk_integrate_rkc",
)


class MechDesc(C.Structure):
    _fields_ = [("n_sp", C.c_int32), ("n_rx", C.c_int32),
                ("reac", C.POINTER(C.c_int32)), ("prod", C.POINTER(C.c_int32)),
                ("lnA", C.POINTER(C.c_double)), ("beta", C.POINTER(C.c_double)),
                ("Ea", C.POINTER(C.c_double)), ("Keq", C.POINTER(C.c_double)),
                ("W", C.POINTER(C.c_double))]


class Options(C.Structure):
    _fields_ = [("max_steps", C.c_int64), ("sr_period", C.c_int32), ("sr_itmax", C.c_int32),
                ("schedule", C.c_int32), ("refill", C.c_int32), ("reserved", C.c_int32 * 6)]


class RKError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rkmi error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32p, dp = C.c_void_p, C.c_int64, C.POINTER(C.c_int32), C.c_void_p
        L.rk_version.restype = C.c_int
        L.rk_last_error.restype = C.c_char_p
        L.rk_problem_create_vdp.argtypes = [C.POINTER(vp)]
        L.rk_problem_create_mass_action.argtypes = [C.POINTER(MechDesc), C.POINTER(vp)]
        L.rk_problem_destroy.argtypes = [vp]
        L.rk_problem_destroy.restype = None
        L.rk_problem_dims.argtypes = [vp, i32p, i32p, i32p]
        L.rk_workspace_bytes.argtypes = [vp, C.c_int32, i64, C.POINTER(Options)]
        L.rk_workspace_bytes.restype = C.c_size_t
        integ = [vp, i64, dp, dp, dp, C.c_double, C.c_double, C.c_double, C.c_double, vp, vp,
                 vp, C.c_size_t, C.POINTER(Options), vp]
        for name in ("rk_integrate_rkck", "rk_integrate_rkc"):
            getattr(L, name).argtypes = integ
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(rc: int):
    if rc != RK_OK:
        raise RKError(rc, lib().rk_last_error().decode())
    return rc
