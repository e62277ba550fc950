"""Pins of the oracle's RKC (Sec. 2.2, Sec. 3.2, Appendix) against closed forms of
the Chebyshev polynomials (mpmath), stability-polynomial theory, the textbook
power iteration, scripted controller cases and an independent integrator."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.integrate import solve_ivp

mp.mp.dps = 40


def cheb_closed(s, w0=None):
    """omega_0, omega_1 and T_j, T_j', T_j'' at omega_0 (j = 0..s) from
    T_j(x) = cosh(j acosh x), in 40-digit arithmetic.  ``w0`` overrides
    omega_0 = 1 + (2/13)/s^2 (e.g. with its double-precision value)."""
    w0 = 1 + mp.mpf(2) / 13 / s ** 2 if w0 is None else mp.mpf(w0)
    th = mp.acosh(w0)
    sh, ch = mp.sinh(th), mp.cosh(th)
    T = [mp.cosh(j * th) for j in range(s + 1)]
    D = [j * mp.sinh(j * th) / sh for j in range(s + 1)]
    E = [j * (j * mp.cosh(j * th) * sh - mp.sinh(j * th) * ch) / sh ** 3 for j in range(s + 1)]
    return w0, D[s] / E[s], T, D, E


def cheb_T(s, x):
    x = mp.mpf(x)
    if abs(x) <= 1:
        return mp.cos(s * mp.acos(x))
    if x > 1:
        return mp.cosh(s * mp.acosh(x))
    return (-1) ** s * mp.cosh(s * mp.acosh(-x))


def P_closed(s, z):
    """RKC stability polynomial P_s(z) = a_s + b_s T_s(omega_0 + omega_1 z)."""
    w0, w1, T, D, E = cheb_closed(s)
    b = E[s] / D[s] ** 2
    a = 1 - b * T[s]
    return a + b * cheb_T(s, w0 + w1 * mp.mpf(z)), (1 + w0) / w1


@pytest.mark.parametrize("s", [2, 3, 7, 50, 400, 2122])
def test_chebyshev_recurrence_vs_closed_form(orc, s):
    co = orc.rkc_coeffs(s)
    assert co["w0"] == pytest.approx(float(1 + mp.mpf(2) / 13 / s ** 2), rel=1e-15)
    # the recurrence is checked at the double omega_0 it was given: near 1 the
    # rounding of omega_0 itself moves T_j by far more than the recurrence does
    w0, w1, T, D, E = cheb_closed(s, co["w0"])
    assert co["w1"] == pytest.approx(float(w1), rel=1e-11)
    for j in range(s + 1):
        assert co["T"][j] == pytest.approx(float(T[j]), rel=1e-11, abs=1e-300)
        assert co["D"][j] == pytest.approx(float(D[j]), rel=1e-11, abs=1e-300)
        assert co["E"][j] == pytest.approx(float(E[j]), rel=1e-10, abs=1e-300)


@pytest.mark.parametrize("s", [2, 3, 4, 9, 30, 120])
def test_stability_polynomial_second_order(s):
    """P_s(0) = P_s'(0) = P_s''(0) = 1: the coefficients define a second-order method."""
    w0, w1, T, D, E = cheb_closed(s)
    b = E[s] / D[s] ** 2
    a = 1 - b * T[s]
    P0 = a + b * T[s]
    P1 = b * w1 * D[s]
    P2 = b * w1 ** 2 * E[s]
    assert abs(P0 - 1) < 1e-30 and abs(P1 - 1) < 1e-30 and abs(P2 - 1) < 1e-30


@pytest.mark.parametrize("s", [2, 3, 5, 10, 37, 150])
def test_one_step_linear_equals_stability_polynomial(orc, s):
    """y' = lam y: one RKC step with s stages gives P_s(h lam) y0, and
    |P_s| <= 1 on the real stability interval [-beta(s), 0]."""
    _, beta = P_closed(s, 0)
    beta = float(beta)
    h, y0 = 0.25, 1.3
    for frac in (0.0, 0.01, 0.1, 0.37, 0.5, 0.81, 0.999):
        z = -frac * beta
        pb = orc.linear([[z / h]])
        F = orc.rhs(pb, None, [y0])
        y1 = orc.rkc_step(pb, None, 0.0, [y0], F, h, s)[0]
        P, _ = P_closed(s, z)
        assert abs(y1 - float(P) * y0) <= 1e-13 * s * abs(y0), (s, frac, y1, float(P) * y0)
        assert abs(y1) <= abs(y0) * (1 + 1e-12)


@pytest.mark.parametrize("s", [2, 3, 6, 25])
def test_stage_times(orc, s):
    """With y' = (y2, 0) every stage is exact: w_j = y + c_j h f, where
    c_1 = c_2 / T_2'(omega_0), c_j = omega_1 T_j''/T_j' (2 <= j <= s-1), c_s = 1
    (Sec. 2.2).  This fixes b_1 (stage 1 sits at mut_1 = b_1 omega_1)."""
    w0, w1, T, D, E = cheb_closed(s)
    c = [None] * (s + 1)
    c[s] = mp.mpf(1)
    for j in range(2, s):
        c[j] = w1 * E[j] / D[j]
    c[1] = c[2] / D[2]
    pb = orc.linear([[0.0, 1.0], [0.0, 0.0]])
    y, h = np.array([0.7, 2.0]), 0.125
    F = orc.rhs(pb, None, y)
    W = orc.rkc_stages(pb, None, 0.0, y, F, h, s)
    for j in range(1, s + 1):
        assert W[j, 1] == pytest.approx(y[1], rel=1e-13)
        assert W[j, 0] - y[0] == pytest.approx(float(c[j]) * h * y[1], rel=1e-12, abs=1e-15)


def test_stage_count_rule_stable_for_all_s():
    """(s^2 - 1)/1.54 <= beta(s) = (1 + omega_0)/omega_1 for s = 2..2122, so the
    stage count of Sec. 2.2 always lands inside the stability interval."""
    mp.mp.dps = 30
    worst = 10.0
    for s in range(2, 2123):
        w0 = 1 + mp.mpf(2) / 13 / s ** 2
        th = mp.acosh(w0)
        sh, ch = mp.sinh(th), mp.cosh(th)
        Ts1 = s * mp.sinh(s * th) / sh
        Ts2 = s * (s * mp.cosh(s * th) * sh - mp.sinh(s * th) * ch) / sh ** 3
        beta = (1 + w0) * Ts2 / Ts1
        worst = min(worst, float(beta / ((s * s - 1) / mp.mpf(1.54))))
    mp.mp.dps = 40
    assert worst >= 1.0


def test_stage_count_function(orc):
    mmax = orc.rkc_mmax(1e-8)
    rng = np.random.default_rng(3)
    for _ in range(300):
        h = 10 ** rng.uniform(-12, -6)
        sig = 10 ** rng.uniform(4, 13)
        m, ho = orc.rkc_stage_count(h, sig, mmax)
        assert 2 <= m <= mmax
        _, beta = P_closed(m, 0) if m < 60 else (None, None)
        if m < mmax:
            assert ho == h
            assert (m - 1) ** 2 <= 1 + 1.54 * h * sig < m * m
            if beta is not None:
                assert h * sig <= float(beta)
        else:
            assert ho <= h
            assert ho == pytest.approx((mmax * mmax - 1) / (1.54 * sig), rel=1e-15)
    # tiny h sigma: two stages
    assert orc.rkc_stage_count(1e-9, 1.0, mmax)[0] == 2


def test_mmax(orc):
    # round(sqrt(rtol / (10 * 2.22e-16))), at least 2
    assert orc.rkc_mmax(1e-8) == 2122
    assert orc.rkc_mmax(1e-6) == 21224
    assert orc.rkc_mmax(1e-13) == 7
    assert orc.rkc_mmax(1e-16) == 2


def test_accept_factor_scripted(orc, consts):
    # first accepted step: min(10, 0.8 / err^(1/3))
    assert orc.rkc_accept_factor(0.5, 0.0, 1.0, 0.0, 0) == pytest.approx(0.8 / 0.5 ** (1 / 3))
    assert orc.rkc_accept_factor(1e-9, 0.0, 1.0, 0.0, 0) == consts["rkc_fac_max"]
    assert orc.rkc_accept_factor(0.0, 0.0, 1.0, 0.0, 0) == 10.0
    # later steps: min(10, 0.8 (h/h_prev) err_prev^(1/3) / err^(2/3))
    got = orc.rkc_accept_factor(0.3, 0.6, 2.0, 1.0, 1)
    assert got == pytest.approx(0.8 * 2.0 * 0.6 ** (1 / 3) / 0.3 ** (2 / 3), rel=1e-14)
    assert orc.rkc_accept_factor(1e-12, 0.6, 2.0, 1.0, 1) == 10.0


# ----------------------------------------------------------------- power method
def _lin_sys(A, seed=0):
    rng = np.random.default_rng(seed)
    y = rng.standard_normal(A.shape[0])
    return y, A @ y


@pytest.mark.parametrize("eigs", [[-1.0, -10.0, -1e3, -1e5],
                                  [-0.5, -3.0, -40.0, -41.0, -900.0, -2500.0],
                                  [-7.0]])
def test_power_method_linear_is_power_iteration(orc, eigs):
    """For f = A y the method is the textbook power iteration on A: the
    estimate is 1.2 times the spectral radius, to its 1% convergence test."""
    from paper_1611_02274_amd.inputs import linear_problem_matrix
    A = linear_problem_matrix(eigs, seed=len(eigs))
    pb = orc.linear(A)
    y, F = _lin_sys(A)
    sig, v, it = orc.spec_rad(pb, None, 0.0, y, F, 1.0, F.copy(), 50)
    rho = max(abs(e) for e in eigs)
    assert it < 50
    assert sig == pytest.approx(1.2 * rho, rel=0.025)
    if len(eigs) > 1:
        # the returned direction is the dominant eigenvector
        lam, vec = np.linalg.eigh(A)
        d = vec[:, np.argmax(np.abs(lam))]
        cosang = abs(v @ d) / np.linalg.norm(v)
        assert cosang > 0.97


def test_power_method_zero_norm_branches(orc):
    A = np.diag([-2.0, -50.0, -3.0])
    pb = orc.linear(A)
    # y = 0 and v = 0: perturbation of size UROUND along the ones vector
    z = np.zeros(3)
    sig, v, it = orc.spec_rad(pb, None, 0.0, z, z, 1.0, z, 50)
    assert sig == pytest.approx(1.2 * 50.0, rel=0.02)
    # y = 0, v != 0
    sig, v, it = orc.spec_rad(pb, None, 0.0, z, z, 1.0, np.array([1.0, 1.0, 1.0]), 50)
    assert sig == pytest.approx(1.2 * 50.0, rel=0.02)
    # y != 0, v = 0: perturbation (1 + sqrt(UROUND)) y
    y = np.array([1.0, 0.5, -2.0])
    sig, v, it = orc.spec_rad(pb, None, 0.0, y, A @ y, 1.0, z, 50)
    assert sig == pytest.approx(1.2 * 50.0, rel=0.02)


def test_power_method_no_convergence_returns_last(orc):
    # two dominant eigenvalues of equal modulus and opposite sign never settle
    # in direction, but the norm ratio is still bounded by the spectral radius
    A = np.diag([-10.0, 10.0])
    pb = orc.linear(A)
    y = np.array([1.0, 1.0])
    sig, v, it = orc.spec_rad(pb, None, 0.0, y, A @ y, 1.0, np.array([1.0, 0.3]), 3)
    assert it <= 3 and 0 < sig <= 1.2 * 10.0 * (1 + 1e-9)


# ----------------------------------------------------------------- whole runs
def test_local_error_order_two(orc):
    pb = orc.vdp()
    mu, y0 = 0.9, np.array([0.8, 0.3])
    errs = []
    for h in (0.04, 0.02, 0.01):
        F = orc.rhs(pb, [mu], y0)
        y1 = orc.rkc_step(pb, [mu], 0.0, y0, F, h, 4)
        ex = solve_ivp(lambda t, y: [y[1], mu * (1 - y[0] ** 2) * y[1] - y[0]], (0, h), y0,
                       method="DOP853", rtol=1e-13, atol=1e-15).y[:, -1]
        errs.append(np.abs(y1 - ex).max())
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(2.7 < s < 3.3 for s in slopes), slopes


def test_adaptive_stiff_linear(orc):
    lam = np.array([-1.0, -1e3, -1e6])
    pb = orc.linear(np.diag(lam))
    y0 = np.array([1.0, 1.0, 1.0])
    rtol, atol = 1e-8, 1e-12
    y1, st, stats, hs, ss = orc.rkc_solve(pb, None, y0, 0.0, 1.0, rtol, atol)
    assert st == orc.OK
    ex = y0 * np.exp(lam * 1.0)
    assert np.all(np.abs(y1 - ex) <= 100 * (atol + rtol * np.abs(y0)))
    # stiffness forces many stages on early steps
    assert stats[orc.ST_MAX_STAGES] > 10
    assert stats[orc.ST_ACCEPT] == len(hs)
    assert abs(hs.sum() - 1.0) < 1e-12


def test_adaptive_vdp(orc):
    pb = orc.vdp()
    mu, y0 = 1.2, np.array([-1.0, 1.5])
    ex = solve_ivp(lambda t, y: [y[1], mu * (1 - y[0] ** 2) * y[1] - y[0]], (0, 4.0), y0,
                   method="DOP853", rtol=1e-13, atol=1e-15).y[:, -1]
    errs = []
    for rtol in (1e-5, 1e-7):
        y1, st, _, _, _ = orc.rkc_solve(pb, [mu], y0, 0.0, 4.0, rtol, rtol)
        assert st == orc.OK
        errs.append(np.abs(y1 - ex).max())
    assert errs[1] < errs[0] and errs[1] < 1e3 * 1e-7


def test_replay_reproduces_solve_bitwise(orc):
    from paper_1611_02274_amd import inputs as I
    net = I.standard_network(13)
    pb = orc.network(net)
    y0, g = I.kinetics_inputs(net, 4, 11)
    for i in range(4):
        y1, st, stats, hs, ss = orc.rkc_solve(pb, g[:, i], y0[:, i], 0.0, 1e-7, 1e-8, 1e-12)
        assert st == orc.OK and len(hs) == stats[orc.ST_ACCEPT]
        yr = orc.rkc_replay(pb, g[:, i], y0[:, i], 0.0, hs, ss)
        assert np.array_equal(yr, y1)


def test_rhs_count_bookkeeping(orc):
    pb = orc.vdp()
    y1, st, stats, hs, ss = orc.rkc_solve(pb, [1.0], [1.0, 0.0], 0.0, 2.0, 1e-6, 1e-8)
    # 1 initial f, 1 initial-step trial, (s - 1) + 1 per attempt, 1 per power iteration
    n_att = stats[orc.ST_ACCEPT] + stats[orc.ST_REJECT]
    assert stats[orc.ST_RHS] >= 2 + 2 * n_att + stats[orc.ST_POW_ITERS]
    assert stats[orc.ST_SR_CALLS] >= 1 + (stats[orc.ST_ACCEPT] - 1) // 25


def test_guards(orc):
    pb = orc.vdp()
    _, st, stats, _, _ = orc.rkc_solve(pb, [1.0], [1.0, 0.0], 0.0, 50.0, 1e-8, 1e-10,
                                       max_steps=7)
    assert st == orc.MAXSTEPS and stats[0] + stats[1] == 7
    pb = orc.linear([[1e300]])
    _, st, _, _, _ = orc.rkc_solve(pb, None, [1.0], 0.0, 1.0, 1e-8, 1e-12)
    assert st in (orc.HMIN, orc.NONFINITE)
