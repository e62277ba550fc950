"""MI355X batched ODE integration: RKCK and RKC over many independent systems.

Thin Python binding of librkmi.so (C ABI in include/rkmi.h): arguments are
checked and marshalled here, every step of the integration runs in the HIP
kernels.  PyTorch provides device memory and the stream.

    import torch, paper_1611_02274_amd as rk
    prob = rk.Problem.network(rk.inputs.standard_network(13))
    y1, status, stats = rk.integrate_rkc(prob, y0, g, 0.0, 1e-6, 1e-8, 1e-12)

with y0 [N, n] and g [P, n] float64 CUDA tensors (struct-of-arrays: row = unknown).
"""
from __future__ import annotations

import ctypes as C

from . import _lib
from ._lib import (RK_METHOD_RKC, RK_METHOD_RKCK, RK_NSTATS, RK_SYS_HMIN, RK_SYS_MAXSTEPS,
                   RK_SYS_NONFINITE, RK_SYS_OK, RKError)

STAT_ACCEPT, STAT_REJECT, STAT_RHS, STAT_SR_CALLS, STAT_POW_ITERS, STAT_MAX_STAGES = range(6)


class Problem:
    """Owns an rk_problem handle."""

    def __init__(self, handle, kind: str, net=None):
        self._h = handle
        self.kind = kind
        self.net = net
        n_eq, n_param, n_theta = C.c_int32(), C.c_int32(), C.c_int32()
        _lib.check(_lib.lib().rk_problem_dims(self._h, C.byref(n_eq), C.byref(n_param),
                                              C.byref(n_theta)))
        self.n_eq, self.n_param, self.n_theta = n_eq.value, n_param.value, n_theta.value

    @classmethod
    def vdp(cls) -> "Problem":
        h = C.c_void_p()
        _lib.check(_lib.lib().rk_problem_create_vdp(C.byref(h)))
        return cls(h, "vdp")

    @classmethod
    def network(cls, net) -> "Problem":
        import numpy as np
        keep = dict(
            reac=np.ascontiguousarray(net.reac, dtype=np.int32),
            prod=np.ascontiguousarray(net.prod, dtype=np.int32),
            lnA=np.ascontiguousarray(net.lnA, dtype=np.float64),
            beta=np.ascontiguousarray(net.beta, dtype=np.float64),
            Ea=np.ascontiguousarray(net.Ea, dtype=np.float64),
            Keq=np.ascontiguousarray(net.Keq, dtype=np.float64),
            W=np.ascontiguousarray(net.W, dtype=np.float64))
        ip, dp = C.POINTER(C.c_int32), C.POINTER(C.c_double)
        d = _lib.MechDesc(net.n_sp, net.n_rx, keep["reac"].ctypes.data_as(ip),
                          keep["prod"].ctypes.data_as(ip), keep["lnA"].ctypes.data_as(dp),
                          keep["beta"].ctypes.data_as(dp), keep["Ea"].ctypes.data_as(dp),
                          keep["Keq"].ctypes.data_as(dp), keep["W"].ctypes.data_as(dp))
        h = C.c_void_p()
        _lib.check(_lib.lib().rk_problem_create_mass_action(C.byref(d), C.byref(h)))
        return cls(h, "mass_action", net)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h is not None and _lib._lib is not None:
            _lib._lib.rk_problem_destroy(h)


def _options(max_steps=None, sr_period=None, sr_itmax=None, schedule=None, refill=None):
    if all(v is None for v in (max_steps, sr_period, sr_itmax, schedule, refill)):
        return None
    o = _lib.Options()
    o.max_steps = int(max_steps or 0)
    o.sr_period = int(sr_period or 0)
    o.sr_itmax = int(sr_itmax or 0)
    o.schedule = int(schedule or 0)
    o.refill = int(refill or 0)
    return o


def _check_tensor(x, name, rows, n, dtype):
    import torch
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if x.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    want = (rows, n) if rows is not None else (n,)
    if tuple(x.shape) != want:
        raise ValueError(f"{name} has shape {tuple(x.shape)}, expected {want}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _integrate(method, problem: Problem, y0, g, t0, t1, rtol, atol, out=None, status=None,
               stats=None, stream=None, **opts):
    import torch
    if y0.dim() != 2:
        raise ValueError("y0 must be [N, n]")
    n = y0.shape[1]
    _check_tensor(y0, "y0", problem.n_eq, n, torch.float64)
    dev = y0.device
    if problem.n_param:
        _check_tensor(g, "g", problem.n_param, n, torch.float64)
        if g.device != dev:
            raise ValueError("g must be on the device of y0")
    if out is None:
        out = torch.empty_like(y0)
    _check_tensor(out, "out", problem.n_eq, n, torch.float64)
    if status is None:
        status = torch.empty(n, dtype=torch.int32, device=dev)
    _check_tensor(status, "status", None, n, torch.int32)
    if stats is None:
        stats = torch.empty((RK_NSTATS, n), dtype=torch.int32, device=dev)
    _check_tensor(stats, "stats", RK_NSTATS, n, torch.int32)
    opt = _options(**opts)
    optp = C.byref(opt) if opt is not None else None
    L = _lib.lib()
    with torch.cuda.device(dev):
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        nws = L.rk_workspace_bytes(problem.handle, method, n, optp)
        ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=dev) if nws else None
        fn = L.rk_integrate_rkck if method == RK_METHOD_RKCK else L.rk_integrate_rkc
        _lib.check(fn(problem.handle, n, y0.data_ptr(), out.data_ptr(),
                      g.data_ptr() if problem.n_param else None, float(t0), float(t1),
                      float(rtol), float(atol), status.data_ptr(), stats.data_ptr(),
                      ws.data_ptr() if ws is not None else None, nws, optp, s.cuda_stream))
    return out, status, stats


def integrate_rkck(problem, y0, g, t0, t1, rtol, atol, **kw):
    """RKCK integration (Sec. 2.1, Sec. 3.1).  Returns (y1, status, stats)."""
    return _integrate(RK_METHOD_RKCK, problem, y0, g, t0, t1, rtol, atol, **kw)


def integrate_rkc(problem, y0, g, t0, t1, rtol, atol, **kw):
    """RKC integration (Sec. 2.2, Sec. 3.2, Appendix).  Returns (y1, status, stats)."""
    return _integrate(RK_METHOD_RKC, problem, y0, g, t0, t1, rtol, atol, **kw)


def version() -> int:
    return _lib.lib().rk_version()


from . import inputs  # noqa: E402  (seeded generators; no integration arithmetic)
