"""ctypes declarations of librkmi.so (include/rkmi.h).

The library is loaded from this package's directory.  There is no fallback: if
it is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# RKMI_LIBRARY names another build of the library (a profiling variant)
LIB_PATH = os.environ.get("RKMI_LIBRARY") or os.path.join(HERE, "librkmi.so")

RK_OK, RK_EINVAL, RK_ENOMEM, RK_EHIP, RK_EUNSUPPORTED, RK_EWORKSPACE = 0, -1, -2, -3, -4, -5
RK_SYS_OK, RK_SYS_NONFINITE, RK_SYS_HMIN, RK_SYS_MAXSTEPS, RK_SYS_TAPE = 0, 1, 2, 3, 4
RK_NSTATS = 6
RK_METHOD_RKCK, RK_METHOD_RKC = 0, 1
RK_SCRATCH_BYTES = 64 << 20   # workspace of rk_integrate_rkc_noalloc per device

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
                ("schedule", C.c_int32), ("refill", C.c_int32), ("cost_order", C.c_int32),
                ("sr_method", C.c_int32), ("group_align", C.c_int32),
                ("reserved", C.c_int32 * 3)]


class BatchSchedule(C.Structure):
    _fields_ = [("mode", C.c_int32), ("waves_per_cu", C.c_int32), ("order", C.c_int32 * 4),
                ("refill", C.c_int32 * 4), ("use_graph", C.c_int32), ("reserved", C.c_int32 * 4)]


RK_BATCH_PERSISTENT, RK_BATCH_PLAIN_INTERLEAVED, RK_BATCH_PLAIN_PER_NETWORK = 0, 1, 2


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
        L.rk_problem_create_pleiades.argtypes = [C.POINTER(vp)]
        L.rk_problem_create_mass_action.argtypes = [C.POINTER(MechDesc), C.POINTER(vp)]
        L.rk_problem_create_mass_action_thermal.argtypes = [C.POINTER(MechDesc), dp, dp, dp,
                                                            C.POINTER(vp)]
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
        L.rk_integrate_rkc_noalloc.argtypes = [vp, i64, dp, dp, dp, C.c_double, C.c_double,
                                               C.c_double, C.c_double, vp, vp,
                                               C.POINTER(Options), vp]
        L.rk_integrate_rkc_noalloc.restype = C.c_int
        L.rk_tape_bytes.argtypes = [vp, i64, i64, C.c_int32]
        L.rk_tape_bytes.restype = C.c_size_t
        L.rk_integrate_rkc_taped.argtypes = [vp, i64, dp, dp, dp, C.c_double, C.c_double,
                                             C.c_double, C.c_double, vp, vp, vp, C.c_size_t,
                                             i64, C.c_int32, C.POINTER(Options), vp]
        L.rk_integrate_rkc_taped.restype = C.c_int
        L.rk_carry_rows.argtypes = [vp]
        L.rk_carry_rows.restype = C.c_size_t
        for name in ("rk_integrate_rkck_carry", "rk_integrate_rkc_carry"):
            getattr(L, name).argtypes = [vp, i64, dp, dp, dp, C.c_double, C.c_double,
                                         C.c_double, C.c_double, vp, vp, dp, vp, C.c_size_t,
                                         C.POINTER(Options), vp]
            getattr(L, name).restype = C.c_int
        L.rk_integrate_rkck_taped.argtypes = L.rk_integrate_rkc_taped.argtypes
        L.rk_integrate_rkck_taped.restype = C.c_int
        L.rk_adjoint_rkck_workspace_bytes.argtypes = [vp, i64, C.c_int32]
        L.rk_adjoint_rkck_workspace_bytes.restype = C.c_size_t
        L.rk_adjoint_rkck.argtypes = [vp, i64, dp, vp, C.c_size_t, i64, C.c_int32, dp, dp, dp,
                                      vp, vp, C.c_size_t, vp]
        L.rk_adjoint_rkck.restype = C.c_int
        L.rk_adjoint_workspace_bytes.argtypes = [vp, i64, C.c_int32, C.c_int32]
        L.rk_adjoint_workspace_bytes.restype = C.c_size_t
        L.rk_adjoint_rkc.argtypes = [vp, i64, dp, vp, C.c_size_t, i64, C.c_int32, C.c_int32, dp,
                                     dp, dp, vp, vp, C.c_size_t, vp]
        L.rk_adjoint_rkc.restype = C.c_int
        L.rk_batch_create.argtypes = [C.POINTER(vp), C.c_int32, C.POINTER(vp)]
        L.rk_batch_create.restype = C.c_int
        L.rk_batch_destroy.argtypes = [vp]
        L.rk_batch_destroy.restype = None
        L.rk_batch_workspace_bytes.argtypes = [vp, C.POINTER(i64), i64, C.POINTER(BatchSchedule)]
        L.rk_batch_workspace_bytes.restype = C.c_size_t
        L.rk_batch_integrate_rkc.argtypes = [vp, C.POINTER(i64), C.POINTER(vp), C.POINTER(vp),
                                             C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), vp,
                                             i64, C.c_double,
                                             C.c_double, C.c_int32, C.c_double, C.c_double,
                                             C.POINTER(Options), C.POINTER(BatchSchedule),
                                             vp, C.c_size_t, vp]
        L.rk_batch_integrate_rkc.restype = C.c_int
        # internal: FP64 vector-ALU throughput probe (benchmark ceilings)
        L.rkmi_peak_threads.argtypes = []
        L.rkmi_peak_threads.restype = i64
        L.rkmi_peak_fp64.argtypes = [C.c_int, i64, dp, C.POINTER(C.c_double), vp]
        L.rkmi_peak_fp64.restype = C.c_int
        _lib = L
    return _lib


def check(rc: int):
    if rc != RK_OK:
        raise RKError(rc, lib().rk_last_error().decode())
    return rc
