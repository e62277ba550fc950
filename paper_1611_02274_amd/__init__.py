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
                   RK_SYS_NONFINITE, RK_SYS_OK, RK_SYS_TAPE, RKError)

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
    def pleiades(cls) -> "Problem":
        h = C.c_void_p()
        _lib.check(_lib.lib().rk_problem_create_pleiades(C.byref(h)))
        return cls(h, "pleiades")

    @classmethod
    def network_thermal(cls, net) -> "Problem":
        """The network with the energy equation (state (T, Y), g = (rho)); net
        must carry its thermodynamics (inputs.thermal_network)."""
        import numpy as np
        keep, d = cls._desc(net)
        th = [np.ascontiguousarray(a, dtype=np.float64) for a in (net.u0, net.cv0, net.cv1)]
        h = C.c_void_p()
        _lib.check(_lib.lib().rk_problem_create_mass_action_thermal(
            C.byref(d), th[0].ctypes.data, th[1].ctypes.data, th[2].ctypes.data, C.byref(h)))
        return cls(h, "mass_action_thermal", net)

    @staticmethod
    def _desc(net):
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
        return keep, d

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
        # at interpreter exit the module globals may already be gone
        h, self._h = getattr(self, "_h", None), None
        try:
            lib = _lib._lib
        except (AttributeError, NameError, TypeError):
            return
        if h is not None and lib is not None:
            lib.rk_problem_destroy(h)


SR_METHODS = {"power": 0, "gershgorin": 1}


def _options(max_steps=None, sr_period=None, sr_itmax=None, schedule=None, refill=None,
             cost_order=None, sr_method=None, group_align=None):
    """rk_options; sr_method (RKC spectral radius): "power" (the nonlinear power
    method, default) or "gershgorin" (the bound of the analytic Jacobian);
    group_align (group schedule): evaluations a group at its error estimate
    waits for another group of its wave (0 default, negative never)."""
    if all(v is None for v in (max_steps, sr_period, sr_itmax, schedule, refill, cost_order,
                               sr_method, group_align)):
        return None
    o = _lib.Options()
    o.max_steps = int(max_steps or 0)
    o.sr_period = int(sr_period or 0)
    o.sr_itmax = int(sr_itmax or 0)
    o.schedule = int(schedule or 0)
    o.refill = int(refill or 0)
    o.cost_order = int(bool(cost_order))
    o.sr_method = SR_METHODS[sr_method] if isinstance(sr_method, str) else int(sr_method or 0)
    o.group_align = int(group_align or 0)
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
               stats=None, stream=None, carry=None, **opts):
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
        gp = g.data_ptr() if problem.n_param else None
        wp = ws.data_ptr() if ws is not None else None
        if carry is None:
            fn = L.rk_integrate_rkck if method == RK_METHOD_RKCK else L.rk_integrate_rkc
            _lib.check(fn(problem.handle, n, y0.data_ptr(), out.data_ptr(), gp, float(t0),
                          float(t1), float(rtol), float(atol), status.data_ptr(),
                          stats.data_ptr(), wp, nws, optp, s.cuda_stream))
        else:
            _check_tensor(carry, "carry", carry_rows(problem), n, torch.float64)
            fn = (L.rk_integrate_rkck_carry if method == RK_METHOD_RKCK
                  else L.rk_integrate_rkc_carry)
            _lib.check(fn(problem.handle, n, y0.data_ptr(), out.data_ptr(), gp, float(t0),
                          float(t1), float(rtol), float(atol), status.data_ptr(),
                          stats.data_ptr(), carry.data_ptr(), wp, nws, optp, s.cuda_stream))
    return out, status, stats


def integrate_rkck(problem, y0, g, t0, t1, rtol, atol, **kw):
    """RKCK integration (Sec. 2.1, Sec. 3.1).  Returns (y1, status, stats)."""
    return _integrate(RK_METHOD_RKCK, problem, y0, g, t0, t1, rtol, atol, **kw)


def integrate_rkc(problem, y0, g, t0, t1, rtol, atol, **kw):
    """RKC integration (Sec. 2.2, Sec. 3.2, Appendix).  Returns (y1, status, stats).
    carry=tensor [carry_rows(problem), n]: the controller state carried between
    calls instead of the restart (zeros at first; updated in place)."""
    return _integrate(RK_METHOD_RKC, problem, y0, g, t0, t1, rtol, atol, **kw)


def carry_rows(problem) -> int:
    """Rows of a carried-state array for `problem` (7 + N)."""
    return int(_lib.lib().rk_carry_rows(problem.handle))


class Tape:
    """Device tape of an RKC or RKCK integration (accepted steps' h and s -- s = 6
    for RKCK -- and the state every ckpt_every accepted steps) for the discrete
    adjoint."""

    def __init__(self, buf, n, max_accepted, ckpt_every, stats, method=RK_METHOD_RKC):
        self.buf, self.n = buf, n
        self.max_accepted, self.ckpt_every = max_accepted, ckpt_every
        self.stats = stats
        self.method = method

    def _offsets(self):
        def a256(x):
            return (x + 255) // 256 * 256
        n, cap = self.n, self.max_accepted
        off_h = a256(4 * n)
        off_s = off_h + a256(8 * cap * n)
        return off_h, off_s

    @property
    def count(self):
        """Accepted steps recorded per system (-1: more than max_accepted)."""
        import torch
        return self.buf[:4 * self.n].view(torch.int32)

    @property
    def h(self):
        """[max_accepted, n] step sizes (rows beyond a system's count unused)."""
        import torch
        off_h, _ = self._offsets()
        n, cap = self.n, self.max_accepted
        return self.buf[off_h:off_h + 8 * cap * n].view(torch.float64).view(cap, n)

    @property
    def s(self):
        """[max_accepted, n] stage counts (rows beyond a system's count unused)."""
        import torch
        _, off_s = self._offsets()
        n, cap = self.n, self.max_accepted
        return self.buf[off_s:off_s + 4 * cap * n].view(torch.int32).view(cap, n)


def integrate_rkc_taped(problem, y0, g, t0, t1, rtol, atol, max_accepted=4096, ckpt_every=16,
                        **kw):
    """RKC integration that also records the tape of the discrete adjoint.
    Returns (y1, status, stats, tape)."""
    return _integrate_taped(RK_METHOD_RKC, problem, y0, g, t0, t1, rtol, atol, max_accepted,
                            ckpt_every, **kw)


def integrate_rkck_taped(problem, y0, g, t0, t1, rtol, atol, max_accepted=4096, ckpt_every=16,
                         **kw):
    """RKCK integration that also records the tape of the discrete adjoint.
    Returns (y1, status, stats, tape)."""
    return _integrate_taped(RK_METHOD_RKCK, problem, y0, g, t0, t1, rtol, atol, max_accepted,
                            ckpt_every, **kw)


def _integrate_taped(method, problem, y0, g, t0, t1, rtol, atol, max_accepted, ckpt_every,
                     out=None, status=None, stats=None, stream=None, **opts):
    import torch
    if y0.dim() != 2:
        raise ValueError("y0 must be [N, n]")
    n = y0.shape[1]
    _check_tensor(y0, "y0", problem.n_eq, n, torch.float64)
    dev = y0.device
    if problem.n_param:
        _check_tensor(g, "g", problem.n_param, n, torch.float64)
    out = torch.empty_like(y0) if out is None else out
    _check_tensor(out, "out", problem.n_eq, n, torch.float64)
    status = torch.empty(n, dtype=torch.int32, device=dev) if status is None else status
    stats = torch.empty((RK_NSTATS, n), dtype=torch.int32, device=dev) if stats is None else stats
    opt = _options(**opts)
    optp = C.byref(opt) if opt is not None else None
    L = _lib.lib()
    nb = L.rk_tape_bytes(problem.handle, n, int(max_accepted), int(ckpt_every))
    if nb == 0 and n > 0:
        raise ValueError("bad tape arguments")
    with torch.cuda.device(dev):
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        buf = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
        fn = L.rk_integrate_rkck_taped if method == RK_METHOD_RKCK else L.rk_integrate_rkc_taped
        _lib.check(fn(
            problem.handle, n, y0.data_ptr(), out.data_ptr(),
            g.data_ptr() if problem.n_param else None, float(t0), float(t1), float(rtol),
            float(atol), status.data_ptr(), stats.data_ptr(), buf.data_ptr(), nb,
            int(max_accepted), int(ckpt_every), optp, s.cuda_stream))
    return out, status, stats, Tape(buf, n, int(max_accepted), int(ckpt_every), stats, method)


def adjoint_rkc(problem, g, tape, dL_dy1, max_stages=None, stream=None):
    """Reverse sweep of the discrete RKC adjoint over `tape`.  Returns
    (dL/dy0 [N, n], per-system dL/dtheta [n_theta, n], status [n])."""
    import torch
    n = tape.n
    _check_tensor(dL_dy1, "dL_dy1", problem.n_eq, n, torch.float64)
    dev = dL_dy1.device
    if max_stages is None:
        max_stages = max(2, int(tape.stats[STAT_MAX_STAGES].max().item())) if n else 2
    L = _lib.lib()
    dy0 = torch.empty_like(dL_dy1)
    dth = torch.empty((max(problem.n_theta, 1), n), dtype=torch.float64, device=dev)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    nws = L.rk_adjoint_workspace_bytes(problem.handle, n, int(max_stages), tape.ckpt_every)
    with torch.cuda.device(dev):
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=dev)
        _lib.check(L.rk_adjoint_rkc(problem.handle, n, g.data_ptr() if problem.n_param else None,
                                    tape.buf.data_ptr(), tape.buf.numel(), tape.max_accepted,
                                    tape.ckpt_every, int(max_stages), dL_dy1.data_ptr(),
                                    dy0.data_ptr(), dth.data_ptr(), st.data_ptr(), ws.data_ptr(),
                                    nws, s.cuda_stream))
    return dy0, dth[:problem.n_theta], st


def adjoint_rkck(problem, g, tape, dL_dy1, stream=None):
    """Reverse sweep of the discrete RKCK adjoint over `tape` (from
    integrate_rkck_taped).  Returns (dL/dy0 [N, n], per-system dL/dtheta
    [n_theta, n], status [n])."""
    import torch
    n = tape.n
    _check_tensor(dL_dy1, "dL_dy1", problem.n_eq, n, torch.float64)
    dev = dL_dy1.device
    L = _lib.lib()
    dy0 = torch.empty_like(dL_dy1)
    dth = torch.empty((max(problem.n_theta, 1), n), dtype=torch.float64, device=dev)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    nws = L.rk_adjoint_rkck_workspace_bytes(problem.handle, n, tape.ckpt_every)
    with torch.cuda.device(dev):
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=dev)
        _lib.check(L.rk_adjoint_rkck(problem.handle, n,
                                     g.data_ptr() if problem.n_param else None,
                                     tape.buf.data_ptr(), tape.buf.numel(), tape.max_accepted,
                                     tape.ckpt_every, dL_dy1.data_ptr(), dy0.data_ptr(),
                                     dth.data_ptr(), st.data_ptr(), ws.data_ptr(), nws,
                                     s.cuda_stream))
    return dy0, dth[:problem.n_theta], st


# Longest tape (accepted steps per system) the autograd functions record
# before giving up on a system: at 2^16 systems of 13 unknowns such a tape
# takes about 80 GB of device memory.
TAPE_LIMIT = 1 << 16


def _autograd_function(method):
    import torch
    taped = integrate_rkck_taped if method == RK_METHOD_RKCK else integrate_rkc_taped
    reverse = adjoint_rkck if method == RK_METHOD_RKCK else adjoint_rkc

    class Adjoint(torch.autograd.Function):
        """y1 = RKC(y0; theta) or RKCK(y0; theta) with the discrete adjoint as its
        backward.  Inputs: y0 [N, n]; g [P, n] (for van der Pol its row 0, mu,
        is the differentiable parameter); lnA [n_rx] or None (networks: the
        shared ln A_j, whose gradient sums the per-system contributions)."""

        @staticmethod
        def forward(ctx, y0, g, lnA, problem, t0, t1, rtol, atol, max_accepted, ckpt_every):
            if problem.kind != "vdp" and g is not None and g.requires_grad:
                raise ValueError("only y0 and lnA are differentiable for a network problem "
                                 "(g = (T, rho) is not): detach g")
            # a system that outruns the tape is recorded again with a tape twice
            # as long, up to TAPE_LIMIT accepted steps per system
            limit = max(max_accepted, TAPE_LIMIT)
            while True:
                y1, status, stats, tape = taped(
                    problem, y0.detach(), g.detach() if g is not None else None, t0, t1, rtol,
                    atol, max_accepted=max_accepted, ckpt_every=ckpt_every)
                if int(tape.count.min().item()) >= 0 or y0.shape[1] == 0:
                    break
                if max_accepted >= limit:
                    raise RuntimeError(f"a system takes more than {max_accepted} accepted "
                                       "steps: no tape for its gradient")
                max_accepted = min(2 * max_accepted, limit)
            ctx.problem, ctx.tape, ctx.has_lnA = problem, tape, lnA is not None
            ctx.save_for_backward(g)
            ctx.mark_non_differentiable(status, stats)
            return y1, status, stats

        @staticmethod
        def backward(ctx, gy1, _gst, _gstats):
            (g,) = ctx.saved_tensors
            dy0, dth, st = reverse(ctx.problem, g, ctx.tape, gy1.contiguous())
            dg = dlnA = None
            if ctx.problem.kind == "vdp" and ctx.needs_input_grad[1]:
                dg = dth
            if ctx.has_lnA and ctx.needs_input_grad[2]:
                dlnA = dth.sum(1)
            return dy0, dg, dlnA, None, None, None, None, None, None, None

    Adjoint.__name__ = "RKCKAdjoint" if method == RK_METHOD_RKCK else "RKCAdjoint"
    return Adjoint


_adjoint_fns = {}
_lnA_problems = {}


def rkc_solve(problem, y0, g, t0, t1, rtol, atol, lnA=None, max_accepted=4096, ckpt_every=16):
    """Differentiable RKC integration: returns (y1, status, stats) with y1 in the
    autograd graph of y0, g (van der Pol: mu) and lnA (networks, [n_rx]; the
    problem's own values when None).  The backward pass is the discrete
    adjoint, checkpointed every ckpt_every accepted steps."""
    return _solve(RK_METHOD_RKC, problem, y0, g, t0, t1, rtol, atol, lnA, max_accepted,
                  ckpt_every)


def rkck_solve(problem, y0, g, t0, t1, rtol, atol, lnA=None, max_accepted=4096, ckpt_every=16):
    """Differentiable RKCK integration, as rkc_solve."""
    return _solve(RK_METHOD_RKCK, problem, y0, g, t0, t1, rtol, atol, lnA, max_accepted,
                  ckpt_every)


def _solve(method, problem, y0, g, t0, t1, rtol, atol, lnA, max_accepted, ckpt_every):
    if method not in _adjoint_fns:
        _adjoint_fns[method] = _autograd_function(method)
    if lnA is not None:
        import dataclasses

        import numpy as np
        if problem.net is None:
            raise ValueError("lnA applies to mass-action networks")
        vals = np.ascontiguousarray(lnA.detach().cpu().numpy(), dtype=np.float64)
        if vals.shape != (problem.net.n_rx,):
            raise ValueError(f"lnA must have shape ({problem.net.n_rx},)")
        if not np.array_equal(vals, problem.net.lnA):
            key = (id(problem), vals.tobytes())
            if key not in _lnA_problems:
                _lnA_problems.clear()
                _lnA_problems[key] = Problem.network(dataclasses.replace(problem.net, lnA=vals))
            problem = _lnA_problems[key]
    return _adjoint_fns[method].apply(y0, g, lnA, problem, t0, t1, rtol, atol, max_accepted,
                                      ckpt_every)


class Batch:
    """Ragged batch over several compiled networks (rk_batch_* in the C ABI):
    RKC over operator-splitting substeps, each a restart, state in place."""

    MODES = {"persistent": _lib.RK_BATCH_PERSISTENT,
             "interleaved": _lib.RK_BATCH_PLAIN_INTERLEAVED,
             "per_network": _lib.RK_BATCH_PLAIN_PER_NETWORK}

    def __init__(self, problems):
        self.problems = list(problems)
        arr = (C.c_void_p * len(self.problems))(*[p.handle.value if hasattr(p.handle, "value")
                                                  else p.handle for p in self.problems])
        h = C.c_void_p()
        _lib.check(_lib.lib().rk_batch_create(arr, len(self.problems), C.byref(h)))
        self._h = h

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        try:
            lib = _lib._lib
        except (AttributeError, NameError, TypeError):
            return
        if h is not None and lib is not None:
            lib.rk_batch_destroy(h)

    @classmethod
    def schedule(cls, mode="persistent", waves_per_cu=0, order=None, refill=None,
                 use_graph=False):
        s = _lib.BatchSchedule()
        s.mode = cls.MODES[mode]
        s.waves_per_cu = int(waves_per_cu)
        for k in range(4):
            s.order[k] = int(order[k]) if order is not None and k < len(order) else -1
            s.refill[k] = int(refill[k]) if refill is not None and k < len(refill) else 0
        s.use_graph = int(bool(use_graph))
        return s

    def integrate_rkc(self, ys, gs, t0, dt, n_substeps, rtol, atol, mode="persistent",
                      waves_per_cu=0, order=None, refill=None, use_graph=False, slot_map=None,
                      status=None, stats=None, stream=None, max_steps=None, carry=None):
        """ys[k] [N_k, n_k] and gs[k] [2, n_k] float64 CUDA tensors per problem,
        integrated in place; status / stats: lists of tensors or None; carry: a
        list of [carry_rows(problem k), n_k] float64 tensors carrying the
        controller state from substep to substep (zeros at first), or None for
        a restart at every substep."""
        import torch
        m = len(self.problems)
        if len(ys) != m or len(gs) != m:
            raise ValueError("one y and one g per problem")
        n = [int(y.shape[1]) for y in ys]
        for k, (p, y, g) in enumerate(zip(self.problems, ys, gs)):
            _check_tensor(y, f"ys[{k}]", p.n_eq, n[k], torch.float64)
            _check_tensor(g, f"gs[{k}]", p.n_param, n[k], torch.float64)
            if carry is not None:
                _check_tensor(carry[k], f"carry[{k}]", carry_rows(p), n[k], torch.float64)
        dev = ys[0].device
        sched = self.schedule(mode, waves_per_cu, order, refill, use_graph)
        n_total = sum(n) if mode == "interleaved" else 0
        if mode == "interleaved":
            _check_tensor(slot_map, "slot_map", None, n_total, torch.int32)
        nn = (C.c_int64 * m)(*n)
        L = _lib.lib()
        nws = L.rk_batch_workspace_bytes(self._h, nn, n_total, C.byref(sched))
        if nws == 0 and sum(n) > 0:
            raise RKError(_lib.RK_EINVAL, L.rk_last_error().decode())

        def ptrs(ts):
            return None if ts is None else (C.c_void_p * m)(*[t.data_ptr() for t in ts])

        opt = _options(max_steps=max_steps)
        with torch.cuda.device(dev):
            s = stream if stream is not None else torch.cuda.current_stream(dev)
            ws = getattr(self, "_ws", None)
            if ws is None or ws.numel() < nws or ws.device != dev:
                # one workspace per batch, reused: a captured graph refers to it
                ws = self._ws = torch.empty(max(nws, 1), dtype=torch.uint8, device=dev)
            _lib.check(L.rk_batch_integrate_rkc(
                self._h, nn, ptrs(ys), ptrs(gs), ptrs(status), ptrs(stats), ptrs(carry),
                slot_map.data_ptr() if mode == "interleaved" else None, n_total, float(t0),
                float(dt), int(n_substeps), float(rtol), float(atol),
                C.byref(opt) if opt is not None else None, C.byref(sched), ws.data_ptr(), nws,
                s.cuda_stream))
        return ys


def version() -> int:
    return _lib.lib().rk_version()


from . import inputs  # noqa: E402  (seeded generators; no integration arithmetic)
