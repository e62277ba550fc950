"""ctypes wrapper of the serial FP64 CPU oracle (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It loads ``oracle/liborc.so`` (building it with gcc if it is absent)
and shares nothing with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

VDP, LINEAR, MASS_ACTION, PLEIADES, MASS_ACTION_THERMAL = 1, 2, 3, 4, 5
OK, NONFINITE, HMIN, MAXSTEPS = 0, 1, 2, 3
NSTATS = 6
ST_ACCEPT, ST_REJECT, ST_RHS, ST_SR_CALLS, ST_POW_ITERS, ST_MAX_STAGES = range(6)
DEFAULT_MAX_STEPS = 10_000_000

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class _Problem(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_eq", C.c_int), ("n_param", C.c_int), ("A", _dp),
                ("n_rx", C.c_int), ("reac", _ip), ("prod", _ip), ("lnA", _dp), ("beta", _dp),
                ("Ea", _dp), ("Keq", _dp), ("W", _dp), ("thermo", _dp), ("sr_method", C.c_int)]


def _d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _i(a):
    return a.ctypes.data_as(_ip) if a is not None else None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.POINTER(_Problem)
        sig = {
            "orc_n_theta": (C.c_int, [P]),
            "orc_rkck_tableau": (None, [_dp, _dp, _dp, _dp, _dp]),
            "orc_rhs": (C.c_int, [P, _dp, C.c_double, _dp, _dp]),
            "orc_rhs_vjp": (C.c_int, [P, _dp, _dp, _dp, _dp, _dp]),
            "orc_rkck_trial": (C.c_int, [P, _dp, C.c_double, _dp, _dp, C.c_double, _dp, _dp]),
            "orc_rkck_error": (C.c_double, [C.c_int, _dp, _dp, _dp, C.c_double, C.c_double,
                                            C.c_double, C.POINTER(C.c_int)]),
            "orc_rkck_control": (C.c_double, [C.c_double, C.c_int, C.c_double, C.c_double,
                                              C.c_double, C.POINTER(C.c_int)]),
            "orc_rkc_coeffs": (C.c_int, [C.c_int, _dp, _dp] + [_dp] * 10),
            "orc_rkc_step": (C.c_int, [P, _dp, C.c_double, _dp, _dp, C.c_double, C.c_int, _dp]),
            "orc_rkc_stages": (C.c_int, [P, _dp, C.c_double, _dp, _dp, C.c_double, C.c_int,
                                         _dp]),
            "orc_gershgorin": (C.c_double, [P, _dp, _dp, _dp]),
            "orc_spec_rad": (C.c_double, [P, _dp, C.c_double, _dp, _dp, C.c_double, _dp, C.c_int,
                                          C.POINTER(C.c_int)]),
            "orc_rkc_mmax": (C.c_int, [C.c_double]),
            "orc_rkc_stage_count": (C.c_int, [C.c_double, C.c_double, C.c_int, _dp]),
            "orc_rkc_accept_factor": (C.c_double, [C.c_double, C.c_double, C.c_double,
                                                   C.c_double, C.c_int]),
            "orc_rkck_solve": (C.c_int, [P, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                         C.c_double, C.c_int64, _ip]),
            "orc_rkc_solve": (C.c_int, [P, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.c_int64, _ip, _dp, _ip, C.c_int64,
                                        C.POINTER(C.c_int64)]),
            "orc_rkc_replay": (C.c_int, [P, _dp, _dp, C.c_double, C.c_int64, _dp, _ip, _dp]),
            "orc_rkc_replay_adjoint": (C.c_int, [P, _dp, _dp, C.c_double, C.c_int64, _dp, _ip,
                                                 _dp, _dp, _dp]),
            "orc_rkck_batch": (C.c_int, [P, C.c_int64, _dp, _dp, _dp, C.c_double, C.c_double,
                                         C.c_double, C.c_double, C.c_int64, _ip, _ip, C.c_int]),
            "orc_rkc_batch": (C.c_int, [P, C.c_int64, _dp, _dp, _dp, C.c_double, C.c_double,
                                        C.c_double, C.c_double, C.c_int64, _ip, _ip, C.c_int]),
            "orc_rkc_adjoint_batch": (C.c_int, [P, C.c_int64, _dp, _dp, C.c_double, C.c_double,
                                                C.c_double, C.c_double, C.c_int64, _dp, _dp, _dp,
                                                _dp, _ip, C.c_int]),
            "orc_rkck_adjoint_batch": (C.c_int, [P, C.c_int64, _dp, _dp, C.c_double, C.c_double,
                                                 C.c_double, C.c_double, C.c_int64, _dp, _dp,
                                                 _dp, _dp, _ip, C.c_int]),
            "orc_rkck_solve_rec": (C.c_int, [P, _dp, _dp, _dp, C.c_double, C.c_double,
                                             C.c_double, C.c_double, C.c_int64, _ip, _dp,
                                             C.c_int64, C.POINTER(C.c_int64)]),
            "orc_rkck_replay": (C.c_int, [P, _dp, _dp, C.c_double, C.c_int64, _dp, _dp]),
            "orc_rkck_replay_adjoint": (C.c_int, [P, _dp, _dp, C.c_double, C.c_int64, _dp, _dp,
                                                  _dp, _dp]),
            "orc_rkck_batch_carry": (C.c_int, [P, C.c_int64, _dp, _dp, _dp, C.c_double,
                                               C.c_double, C.c_double, C.c_double, C.c_int64,
                                               _ip, _ip, _dp, C.c_int]),
            "orc_rkc_batch_carry": (C.c_int, [P, C.c_int64, _dp, _dp, _dp, C.c_double,
                                              C.c_double, C.c_double, C.c_double, C.c_int64,
                                              _ip, _ip, _dp, C.c_int]),
            "orc_rkc_solve_trace": (C.c_int, [P, _dp, _dp, _dp, C.c_double, C.c_double,
                                              C.c_double, C.c_double, C.c_int64, _ip,
                                              C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]),
            "orc_rkc_replay_jvp_cs": (C.c_int, [P, _dp, _dp, C.c_double, C.c_int64, _dp, _ip,
                                                _dp, _dp, _dp, _dp]),
            "orc_rkck_replay_jvp_cs": (C.c_int, [P, _dp, _dp, C.c_double, C.c_int64, _dp, _dp,
                                                 _dp, _dp, _dp]),
            "orc_max_threads": (C.c_int, []),
            "orc_cr_exp": (C.c_double, [C.c_double]),
            "orc_cr_log": (C.c_double, [C.c_double]),
            "orc_cr_pow": (C.c_double, [C.c_double, C.c_double]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class Problem:
    """A problem description for the oracle; keeps its arrays alive."""

    def __init__(self, kind, n_eq, n_param, A=None, net=None, lnA=None, sr_method=0):
        self._keep = []
        s = _Problem()
        s.kind, s.n_eq, s.n_param = kind, n_eq, n_param
        s.sr_method = sr_method
        self.sr_method = sr_method
        if A is not None:
            A = np.ascontiguousarray(A, dtype=np.float64)
            self._keep.append(A)
            s.A = _d(A)
        self.net = net
        if net is not None:
            arrs = dict(
                reac=np.ascontiguousarray(net.reac, dtype=np.int32),
                prod=np.ascontiguousarray(net.prod, dtype=np.int32),
                lnA=np.ascontiguousarray(net.lnA if lnA is None else lnA, dtype=np.float64),
                beta=np.ascontiguousarray(net.beta, dtype=np.float64),
                Ea=np.ascontiguousarray(net.Ea, dtype=np.float64),
                Keq=np.ascontiguousarray(net.Keq, dtype=np.float64),
                W=np.ascontiguousarray(net.W, dtype=np.float64))
            self._keep.extend(arrs.values())
            s.n_rx = net.n_rx
            s.reac, s.prod = _i(arrs["reac"]), _i(arrs["prod"])
            s.lnA, s.beta, s.Ea = _d(arrs["lnA"]), _d(arrs["beta"]), _d(arrs["Ea"])
            s.Keq, s.W = _d(arrs["Keq"]), _d(arrs["W"])
            self.lnA = arrs["lnA"]
            if kind == MASS_ACTION_THERMAL:
                th = np.ascontiguousarray(np.stack([net.u0, net.cv0, net.cv1]), dtype=np.float64)
                self._keep.append(th)
                s.thermo = _d(th)
        self.s = s
        self.n_eq, self.n_param = n_eq, n_param

    @property
    def ptr(self):
        return C.byref(self.s)

    @property
    def n_theta(self):
        return lib().orc_n_theta(self.ptr)

    def with_lnA(self, lnA):
        return Problem(MASS_ACTION, self.n_eq, self.n_param, net=self.net, lnA=lnA,
                       sr_method=self.sr_method)

    def gershgorin(self, g, y):
        """(sigma, J): the Gershgorin bound and the analytic Jacobian df/dy at
        y (one system, g its parameters)."""
        g = np.ascontiguousarray(g, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        J = np.zeros((self.n_eq, self.n_eq))
        sig = lib().orc_gershgorin(self.ptr, _d(g), _d(y), _d(J))
        if sig < 0.0:
            raise ValueError("no analytic Jacobian for this problem")
        return sig, J


# RKC spectral radius: the nonlinear power method (Appendix) or the Gershgorin
# bound of the analytic Jacobian
SR_POWER, SR_GERSHGORIN = 0, 1


def vdp(sr_method=SR_POWER):
    return Problem(VDP, 2, 1, sr_method=sr_method)


def linear(A):
    A = np.asarray(A, dtype=np.float64)
    return Problem(LINEAR, A.shape[0], 0, A=A)


def network(net, sr_method=SR_POWER):
    return Problem(MASS_ACTION, net.n_sp, 2, net=net, sr_method=sr_method)


def network_thermal(net):
    """The network with the energy equation: state (T, Y_1..Y_N), g = (rho)."""
    return Problem(MASS_ACTION_THERMAL, net.n_sp + 1, 1, net=net)


def pleiades():
    """The seven-body Pleiades problem (28 unknowns, no per-system parameters)."""
    return Problem(PLEIADES, 28, 0)


def _vec(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    if n is not None:
        assert a.size == n
    return a


def _g(pb, g):
    return _vec(g if g is not None and np.size(g) else np.zeros(1))


# ---------------------------------------------------------------- pieces
def rkck_tableau():
    a, b, c, cs, e = (np.zeros(6), np.zeros(36), np.zeros(6), np.zeros(6), np.zeros(6))
    lib().orc_rkck_tableau(_d(a), _d(b), _d(c), _d(cs), _d(e))
    return a, b.reshape(6, 6), c, cs, e


def rhs(pb, g, y, t=0.0):
    y = _vec(y, pb.n_eq)
    f = np.zeros(pb.n_eq)
    assert lib().orc_rhs(pb.ptr, _d(_g(pb, g)), t, _d(y), _d(f)) == 0
    return f


def rhs_vjp(pb, g, y, u):
    y, u = _vec(y, pb.n_eq), _vec(u, pb.n_eq)
    jtu = np.zeros(pb.n_eq)
    th = np.zeros(max(pb.n_theta, 1))
    assert lib().orc_rhs_vjp(pb.ptr, _d(_g(pb, g)), _d(y), _d(u), _d(jtu), _d(th)) == 0
    return jtu, th[:pb.n_theta]


def rkck_trial(pb, g, t, y, F, h):
    y, F = _vec(y, pb.n_eq), _vec(F, pb.n_eq)
    yt, ye = np.zeros(pb.n_eq), np.zeros(pb.n_eq)
    assert lib().orc_rkck_trial(pb.ptr, _d(_g(pb, g)), t, _d(y), _d(F), h, _d(yt), _d(ye)) == 0
    return yt, ye


def rkck_error(y, F, yerr, h, rtol, atol):
    y, F, yerr = _vec(y), _vec(F), _vec(yerr)
    nan = C.c_int(0)
    e = lib().orc_rkck_error(y.size, _d(y), _d(F), _d(yerr), h, rtol, atol, C.byref(nan))
    return e, nan.value


def rkck_control(err, nan_flag, h, hmin, hmax):
    acc = C.c_int(0)
    hn = lib().orc_rkck_control(err, int(nan_flag), h, hmin, hmax, C.byref(acc))
    return hn, acc.value


def rkc_coeffs(s):
    w0, w1 = C.c_double(), C.c_double()
    names = ["T", "D", "E", "b", "a", "mu", "nu", "mut", "gt", "c"]
    arrs = {k: np.zeros(s + 1) for k in names}
    rc = lib().orc_rkc_coeffs(s, C.byref(w0), C.byref(w1), *[_d(arrs[k]) for k in names])
    assert rc == 0
    arrs["w0"], arrs["w1"] = w0.value, w1.value
    return arrs


def rkc_step(pb, g, t, y, F, h, s):
    y, F = _vec(y, pb.n_eq), _vec(F, pb.n_eq)
    out = np.zeros(pb.n_eq)
    assert lib().orc_rkc_step(pb.ptr, _d(_g(pb, g)), t, _d(y), _d(F), h, s, _d(out)) == 0
    return out


def rkc_stages(pb, g, t, y, F, h, s):
    y, F = _vec(y, pb.n_eq), _vec(F, pb.n_eq)
    W = np.zeros((s + 1, pb.n_eq))
    assert lib().orc_rkc_stages(pb.ptr, _d(_g(pb, g)), t, _d(y), _d(F), h, s, _d(W)) == 0
    return W


def spec_rad(pb, g, t, y, F, hmax, v, itmax=50):
    y, F = _vec(y, pb.n_eq), _vec(F, pb.n_eq)
    v = _vec(v, pb.n_eq).copy()
    it = C.c_int(0)
    sig = lib().orc_spec_rad(pb.ptr, _d(_g(pb, g)), t, _d(y), _d(F), hmax, _d(v), itmax,
                             C.byref(it))
    return sig, v, it.value


def rkc_mmax(rtol):
    return lib().orc_rkc_mmax(rtol)


def rkc_stage_count(h, sigma, mmax):
    ho = C.c_double()
    m = lib().orc_rkc_stage_count(h, sigma, mmax, C.byref(ho))
    return m, ho.value


def rkc_accept_factor(err, err_prev, h, h_prev, have_prev):
    return lib().orc_rkc_accept_factor(err, err_prev, h, h_prev, int(have_prev))


# ---------------------------------------------------------------- one system
def rkck_solve(pb, g, y0, t0, t1, rtol, atol, max_steps=DEFAULT_MAX_STEPS):
    y0 = _vec(y0, pb.n_eq)
    y1 = np.zeros(pb.n_eq)
    st = np.zeros(NSTATS, dtype=np.int32)
    rc = lib().orc_rkck_solve(pb.ptr, _d(_g(pb, g)), _d(y0), _d(y1), t0, t1, rtol, atol,
                              max_steps, _i(st))
    assert rc >= 0, rc
    return y1, rc, st


def rkc_solve(pb, g, y0, t0, t1, rtol, atol, max_steps=DEFAULT_MAX_STEPS, rec_cap=1 << 20):
    """Returns (y1, status, stats, h_steps, s_steps) with the accepted steps."""
    y0 = _vec(y0, pb.n_eq)
    y1 = np.zeros(pb.n_eq)
    st = np.zeros(NSTATS, dtype=np.int32)
    rh = np.zeros(rec_cap)
    rs = np.zeros(rec_cap, dtype=np.int32)
    nrec = C.c_int64(0)
    rc = lib().orc_rkc_solve(pb.ptr, _d(_g(pb, g)), _d(y0), _d(y1), t0, t1, rtol, atol,
                             max_steps, _i(st), _d(rh), _i(rs), rec_cap, C.byref(nrec))
    assert rc >= 0, rc
    n = min(nrec.value, rec_cap)
    return y1, rc, st, rh[:n].copy(), rs[:n].copy()


# One attempted RKC step (orc_rkc_attempt).
ATTEMPT = np.dtype([("t", np.float64), ("h_want", np.float64), ("h", np.float64),
                    ("sigma", np.float64), ("err", np.float64), ("nstep", np.int64),
                    ("n_sr", np.int64), ("m", np.int32), ("accepted", np.int32)])


def rkc_trace(pb, g, y0, t0, t1, rtol, atol, max_steps=DEFAULT_MAX_STEPS, cap=1 << 18):
    """RKC as rkc_solve; returns (y1, status, stats, trace) with one record of
    ATTEMPT per attempted step."""
    y0 = _vec(y0, pb.n_eq)
    y1 = np.zeros(pb.n_eq)
    st = np.zeros(NSTATS, dtype=np.int32)
    tr = np.zeros(cap, dtype=ATTEMPT)
    n = C.c_int64(0)
    rc = lib().orc_rkc_solve_trace(pb.ptr, _d(_g(pb, g)), _d(y0), _d(y1), t0, t1, rtol, atol,
                                   max_steps, _i(st), tr.ctypes.data_as(C.c_void_p), cap,
                                   C.byref(n))
    assert rc >= 0, rc
    assert n.value <= cap
    return y1, rc, st, tr[:n.value].copy()


def rkc_replay_jvp_cs(pb, g, y0, t0, h, s, w, dy0, dtheta=None):
    """Complex-step derivative of w . y(t1) along (dy0, dtheta) for the replayed
    RKC steps (h, s)."""
    y0, w, dy0, h = _vec(y0, pb.n_eq), _vec(w, pb.n_eq), _vec(dy0, pb.n_eq), _vec(h)
    s = np.ascontiguousarray(s, dtype=np.int32)
    dth = _vec(dtheta, pb.n_theta) if dtheta is not None else None
    out = C.c_double()
    assert lib().orc_rkc_replay_jvp_cs(pb.ptr, _d(_g(pb, g)), _d(y0), t0, h.size, _d(h), _i(s),
                                       _d(w), _d(dy0), _d(dth), C.byref(out)) == 0
    return out.value


def rkck_replay_jvp_cs(pb, g, y0, t0, h, w, dy0, dtheta=None):
    """Complex-step derivative of w . y(t1) along (dy0, dtheta) for the replayed
    RKCK steps h."""
    y0, w, dy0, h = _vec(y0, pb.n_eq), _vec(w, pb.n_eq), _vec(dy0, pb.n_eq), _vec(h)
    dth = _vec(dtheta, pb.n_theta) if dtheta is not None else None
    out = C.c_double()
    assert lib().orc_rkck_replay_jvp_cs(pb.ptr, _d(_g(pb, g)), _d(y0), t0, h.size, _d(h),
                                        _d(w), _d(dy0), _d(dth), C.byref(out)) == 0
    return out.value


def rkck_solve_rec(pb, g, y0, t0, t1, rtol, atol, max_steps=DEFAULT_MAX_STEPS, rec_cap=1 << 20):
    """RKCK as rkck_solve; returns (y1, status, stats, h_steps) with the accepted steps."""
    y0 = _vec(y0, pb.n_eq)
    y1 = np.zeros(pb.n_eq)
    st = np.zeros(NSTATS, dtype=np.int32)
    rh = np.zeros(rec_cap)
    nrec = C.c_int64(0)
    rc = lib().orc_rkck_solve_rec(pb.ptr, _d(_g(pb, g)), _d(y0), _d(y1), t0, t1, rtol, atol,
                                  max_steps, _i(st), _d(rh), rec_cap, C.byref(nrec))
    assert rc >= 0, rc
    return y1, rc, st, rh[:min(nrec.value, rec_cap)].copy()


def rkck_replay(pb, g, y0, t0, h):
    y0, h = _vec(y0, pb.n_eq), _vec(h)
    y1 = np.zeros(pb.n_eq)
    assert lib().orc_rkck_replay(pb.ptr, _d(_g(pb, g)), _d(y0), t0, h.size, _d(h), _d(y1)) == 0
    return y1


def rkck_replay_adjoint(pb, g, y0, t0, h, w):
    y0, w, h = _vec(y0, pb.n_eq), _vec(w, pb.n_eq), _vec(h)
    dy0 = np.zeros(pb.n_eq)
    dth = np.zeros(max(pb.n_theta, 1))
    assert lib().orc_rkck_replay_adjoint(pb.ptr, _d(_g(pb, g)), _d(y0), t0, h.size, _d(h),
                                         _d(w), _d(dy0), _d(dth)) == 0
    return dy0, dth[:pb.n_theta]


def rkc_replay(pb, g, y0, t0, h, s):
    y0 = _vec(y0, pb.n_eq)
    h = _vec(h)
    s = np.ascontiguousarray(s, dtype=np.int32)
    y1 = np.zeros(pb.n_eq)
    assert lib().orc_rkc_replay(pb.ptr, _d(_g(pb, g)), _d(y0), t0, h.size, _d(h), _i(s),
                                _d(y1)) == 0
    return y1


def rkc_replay_adjoint(pb, g, y0, t0, h, s, w):
    y0, w = _vec(y0, pb.n_eq), _vec(w, pb.n_eq)
    h = _vec(h)
    s = np.ascontiguousarray(s, dtype=np.int32)
    dy0 = np.zeros(pb.n_eq)
    dth = np.zeros(max(pb.n_theta, 1))
    assert lib().orc_rkc_replay_adjoint(pb.ptr, _d(_g(pb, g)), _d(y0), t0, h.size, _d(h),
                                        _i(s), _d(w), _d(dy0), _d(dth)) == 0
    return dy0, dth[:pb.n_theta]


# ---------------------------------------------------------------- batches
def _batch(fn, pb, y0, g, t0, t1, rtol, atol, max_steps, n_threads):
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    n = y0.shape[1]
    g = np.ascontiguousarray(g, dtype=np.float64) if g is not None else np.zeros((0, n))
    assert y0.shape[0] == pb.n_eq and g.shape[0] >= pb.n_param
    y1 = np.zeros_like(y0)
    status = np.zeros(n, dtype=np.int32)
    stats = np.zeros((NSTATS, n), dtype=np.int32)
    rc = fn(pb.ptr, n, _d(y0), _d(g) if g.size else None, _d(y1), t0, t1, rtol, atol,
            max_steps, _i(status), _i(stats), n_threads)
    assert rc == 0, rc
    return y1, status, stats


CARRY_ROWS = 7      # valid, h, h_prev, err_prev, sigma, nstep, have_prev; then v [N]


def carry_init(pb, n):
    """A carried-state array [CARRY_ROWS + N, n] asking every system to restart."""
    return np.zeros((CARRY_ROWS + pb.n_eq, n))


def _batch_carry(fn, pb, y0, g, carry, t0, t1, rtol, atol, max_steps, n_threads):
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    n = y0.shape[1]
    g = np.ascontiguousarray(g, dtype=np.float64) if g is not None else np.zeros((0, n))
    assert carry.shape == (CARRY_ROWS + pb.n_eq, n) and carry.flags.c_contiguous
    assert carry.dtype == np.float64
    y1 = np.zeros_like(y0)
    status = np.zeros(n, dtype=np.int32)
    stats = np.zeros((NSTATS, n), dtype=np.int32)
    rc = fn(pb.ptr, n, _d(y0), _d(g) if g.size else None, _d(y1), t0, t1, rtol, atol,
            max_steps, _i(status), _i(stats), _d(carry), n_threads)
    assert rc == 0, rc
    return y1, status, stats


def rkck_batch_carry(pb, y0, g, carry, t0, t1, rtol, atol, max_steps=DEFAULT_MAX_STEPS,
                     n_threads=0):
    """RKCK with the controller state carried in `carry` (updated in place)."""
    return _batch_carry(lib().orc_rkck_batch_carry, pb, y0, g, carry, t0, t1, rtol, atol,
                        max_steps, n_threads)


def rkc_batch_carry(pb, y0, g, carry, t0, t1, rtol, atol, max_steps=DEFAULT_MAX_STEPS,
                    n_threads=0):
    """RKC with the controller state carried in `carry` (updated in place)."""
    return _batch_carry(lib().orc_rkc_batch_carry, pb, y0, g, carry, t0, t1, rtol, atol,
                        max_steps, n_threads)


def rkck_batch(pb, y0, g, t0, t1, rtol, atol, max_steps=DEFAULT_MAX_STEPS, n_threads=0):
    return _batch(lib().orc_rkck_batch, pb, y0, g, t0, t1, rtol, atol, max_steps, n_threads)


def rkc_batch(pb, y0, g, t0, t1, rtol, atol, max_steps=DEFAULT_MAX_STEPS, n_threads=0):
    return _batch(lib().orc_rkc_batch, pb, y0, g, t0, t1, rtol, atol, max_steps, n_threads)


def rkc_adjoint_batch(pb, y0, g, w, t0, t1, rtol, atol, max_steps=DEFAULT_MAX_STEPS,
                      n_threads=0):
    """Forward RKC from y0 and the discrete adjoint of its accepted steps for
    L = sum(w * y(t1)); returns (y1, dL/dy0 [N, n], dL/dtheta [n_theta, n], status)."""
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = y0.shape[1]
    y1, dy0 = np.zeros_like(y0), np.zeros_like(y0)
    dth = np.zeros((max(pb.n_theta, 1), n))
    status = np.zeros(n, dtype=np.int32)
    rc = lib().orc_rkc_adjoint_batch(pb.ptr, n, _d(y0), _d(g), t0, t1, rtol, atol, max_steps,
                                     _d(w), _d(y1), _d(dy0), _d(dth), _i(status), n_threads)
    assert rc == 0, rc
    return y1, dy0, dth[:pb.n_theta], status


def rkck_adjoint_batch(pb, y0, g, w, t0, t1, rtol, atol, max_steps=DEFAULT_MAX_STEPS,
                       n_threads=0):
    """Forward RKCK and the discrete adjoint of its accepted steps, as
    rkc_adjoint_batch."""
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = y0.shape[1]
    y1, dy0 = np.zeros_like(y0), np.zeros_like(y0)
    dth = np.zeros((max(pb.n_theta, 1), n))
    status = np.zeros(n, dtype=np.int32)
    rc = lib().orc_rkck_adjoint_batch(pb.ptr, n, _d(y0), _d(g), t0, t1, rtol, atol, max_steps,
                                      _d(w), _d(y1), _d(dy0), _d(dth), _i(status), n_threads)
    assert rc == 0, rc
    return y1, dy0, dth[:pb.n_theta], status


def cr_exp(x):
    return lib().orc_cr_exp(float(x))


def cr_log(x):
    return lib().orc_cr_log(float(x))


def cr_pow(x, y):
    return lib().orc_cr_pow(float(x), float(y))


def max_threads():
    return lib().orc_max_threads()
