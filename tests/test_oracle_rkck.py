"""Pins of the oracle's RKCK (Sec. 2.1 / Sec. 3.1) against the paper's Table 1,
Runge-Kutta order theory, closed forms and an independent library integrator."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import solve_ivp

pytestmark = pytest.mark.filterwarnings("ignore")


# ----------------------------------------------------------------- Table 1
def _order_conditions(A, b, c, order):
    """Butcher order conditions up to `order` (trees of order <= 5), exact."""
    n = len(b)

    def dot(u, v):
        return sum(x * y for x, y in zip(u, v))

    def mat(v):
        return [sum(A[i][j] * v[j] for j in range(n)) for i in range(n)]

    def pw(v, k):
        return [x ** k for x in v]

    def mul(u, v):
        return [x * y for x, y in zip(u, v)]

    one = [Fraction(1)] * n
    Ac = mat(c)
    conds = [(dot(b, one), Fraction(1))]
    if order >= 2:
        conds += [(dot(b, c), Fraction(1, 2))]
    if order >= 3:
        conds += [(dot(b, pw(c, 2)), Fraction(1, 3)), (dot(b, Ac), Fraction(1, 6))]
    if order >= 4:
        conds += [(dot(b, pw(c, 3)), Fraction(1, 4)), (dot(b, mul(c, Ac)), Fraction(1, 8)),
                  (dot(b, mat(pw(c, 2))), Fraction(1, 12)), (dot(b, mat(Ac)), Fraction(1, 24))]
    if order >= 5:
        conds += [(dot(b, pw(c, 4)), Fraction(1, 5)),
                  (dot(b, mul(pw(c, 2), Ac)), Fraction(1, 10)),
                  (dot(b, pw(Ac, 2)), Fraction(1, 20)),
                  (dot(b, mul(c, mat(pw(c, 2)))), Fraction(1, 15)),
                  (dot(b, mul(c, mat(Ac))), Fraction(1, 30)),
                  (dot(b, mat(pw(c, 3))), Fraction(1, 20)),
                  (dot(b, mat(mul(c, Ac))), Fraction(1, 40)),
                  (dot(b, mat(mat(pw(c, 2)))), Fraction(1, 60)),
                  (dot(b, mat(mat(Ac))), Fraction(1, 120))]
    return conds


def _full_A(b_rows):
    A = [[Fraction(0)] * 6 for _ in range(6)]
    for i in range(6):
        for j in range(5):
            A[i][j] = b_rows[i][j]
    return A


def test_table1_row_sums(table1):
    a, b, _, _ = table1
    for i in range(6):
        assert sum(b[i]) == a[i]


def test_table1_fifth_order(table1):
    a, b, c, _ = table1
    conds = _order_conditions(_full_A(b), c, a, 5)
    assert len(conds) == 17
    for got, want in conds:
        assert got == want


def test_table1_embedded_fourth_order(table1):
    a, b, _, cs = table1
    A = _full_A(b)
    conds4 = _order_conditions(A, cs, a, 4)
    assert len(conds4) == 8
    for got, want in conds4:
        assert got == want
    # a genuinely fourth-order companion: it must miss some fifth-order condition
    conds5 = _order_conditions(A, cs, a, 5)[8:]
    assert sum(got != want for got, want in conds5) > 0


def test_oracle_tableau_is_table1(orc, table1):
    a, b, c, cs = table1
    oa, ob, oc, ocs, oe = orc.rkck_tableau()
    for i in range(6):
        assert oa[i] == float(a[i])
        assert oc[i] == float(c[i])
        assert ocs[i] == float(cs[i])
        # error weights: nearest double of the exact difference c_i - c*_i
        assert oe[i] == float(c[i] - cs[i])
        for j in range(5):
            assert ob[i, j] == float(b[i][j])


def _stability_coeffs(table1, weights):
    """gamma_k of R(z) = sum_k gamma_k z^k: gamma_0 = 1, gamma_k = w^T A^(k-1) 1."""
    a, b, _, _ = table1
    A = _full_A(b)
    v = [Fraction(1)] * 6
    g = [Fraction(1)]
    for _ in range(6):
        g.append(sum(w * x for w, x in zip(weights, v)))
        v = [sum(A[i][j] * v[j] for j in range(6)) for i in range(6)]
    return g


def test_stability_polynomial_coefficients(table1):
    _, _, c, cs = table1
    g = _stability_coeffs(table1, c)
    for k in range(6):
        assert g[k] == Fraction(1, math.factorial(k))
    assert g[6] == Fraction(1, 800)
    gs = _stability_coeffs(table1, cs)
    for k in range(5):
        assert gs[k] == Fraction(1, math.factorial(k))
    assert gs[6] == Fraction(1771, 1638400)


@pytest.mark.parametrize("z", [-0.05, -0.7, -2.5, 0.3, 1.2])
def test_one_step_linear_matches_stability_function(orc, table1, z):
    """y' = lam y: one trial step gives R(z) y0 and the error estimate
    (R - R*)(z) y0, z = h lam, with R, R* from Table 1 (closed form)."""
    _, _, c, cs = table1
    g5, g4 = _stability_coeffs(table1, c), _stability_coeffs(table1, cs)
    h, y0 = 0.4, 1.7
    lam = z / h
    pb = orc.linear([[lam]])
    F = orc.rhs(pb, None, [y0])
    yt, ye = orc.rkck_trial(pb, None, 0.0, [y0], F, h)
    R = sum(float(g) * z ** k for k, g in enumerate(g5))
    Rs = sum(float(g) * z ** k for k, g in enumerate(g4))
    scale = sum(abs(float(g) * z ** k) for k, g in enumerate(g5)) * abs(y0)
    assert abs(yt[0] - R * y0) <= 8 * np.finfo(float).eps * scale
    assert abs(ye[0] - (R - Rs) * y0) <= 8 * np.finfo(float).eps * scale


def _vdp_exact(y0, mu, T):
    sol = solve_ivp(lambda t, y: [y[1], mu * (1 - y[0] ** 2) * y[1] - y[0]], (0, T), y0,
                    method="DOP853", rtol=1e-13, atol=1e-15)
    return sol.y[:, -1]


def test_local_error_orders_vdp(orc):
    """Fixed single steps on van der Pol: local error of the fifth-order
    solution falls as h^6, of the embedded solution as h^5."""
    pb = orc.vdp()
    mu, y0 = 1.3, np.array([1.1, -0.4])
    hs = [0.2, 0.1, 0.05]
    e5, e4 = [], []
    for h in hs:
        F = orc.rhs(pb, [mu], y0)
        yt, ye = orc.rkck_trial(pb, [mu], 0.0, y0, F, h)
        ex = _vdp_exact(y0, mu, h)
        e5.append(np.abs(yt - ex).max())
        e4.append(np.abs((yt - ye) - ex).max())
    s5 = [math.log2(e5[i] / e5[i + 1]) for i in range(2)]
    s4 = [math.log2(e4[i] / e4[i + 1]) for i in range(2)]
    assert all(5.5 < s < 6.6 for s in s5), s5
    assert all(4.5 < s < 5.6 for s in s4), s4


# ----------------------------------------------------------------- error/controller
def test_error_norm_hand_example(orc):
    # err = max_i |yerr_i / (|y_i| + |h F_i| + atol/rtol)| / rtol
    y, F, yerr, h = [2.0, -1.0], [4.0, 10.0], [3e-8, -2e-8], 0.5
    rtol, atol = 1e-6, 1e-6   # delta = 1
    # component 0: 3e-8 / (2 + 2 + 1) = 6e-9 ; component 1: 2e-8 / (1 + 5 + 1)
    err, nan = orc.rkck_error(y, F, yerr, h, rtol, atol)
    assert nan == 0
    assert err == pytest.approx(6e-9 / 1e-6, rel=1e-15)
    err, nan = orc.rkck_error(y, F, [float("nan"), 1e-9], h, rtol, atol)
    assert nan == 1
    # atol = 0: delta is the tiny constant 1e-30
    err, _ = orc.rkck_error([0.0], [0.0], [1e-40], 1.0, 1e-6, 0.0)
    assert err == pytest.approx(1e-40 / 1e-30 / 1e-6, rel=1e-12)


def test_controller_scripted(orc, consts):
    S, pg, ps = consts["rkck_safety"], consts["rkck_pgrow"], consts["rkck_pshrnk"]
    errcon = consts["rkck_errcon"]
    hmin, hmax = 1e-20, 10.0
    # accepted, moderate error: S h err^(-1/5)
    h, acc = orc.rkck_control(0.5, 0, 1.0, hmin, hmax)
    assert acc == 1 and h == pytest.approx(S * 0.5 ** pg, rel=1e-15)
    # accepted, tiny error: growth by five
    h, acc = orc.rkck_control(errcon / 2, 0, 1.0, hmin, hmax)
    assert acc == 1 and h == 5.0
    # accepted, zero error
    h, acc = orc.rkck_control(0.0, 0, 3.0, hmin, hmax)
    assert acc == 1 and h == hmax
    # accepted exactly at the threshold err = 1
    h, acc = orc.rkck_control(1.0, 0, 1.0, hmin, hmax)
    assert acc == 1 and h == pytest.approx(S)
    # rejected: S h err^(-1/4), but never below a tenth
    h, acc = orc.rkck_control(2.0, 0, 1.0, hmin, hmax)
    assert acc == 0 and h == pytest.approx(S * 2.0 ** ps, rel=1e-15)
    h, acc = orc.rkck_control(1e8, 0, 1.0, hmin, hmax)
    assert acc == 0 and h == pytest.approx(0.1)
    # NaN error or NaN component: rejected, cut by ten
    h, acc = orc.rkck_control(float("nan"), 0, 1.0, hmin, hmax)
    assert acc == 0 and h == pytest.approx(0.1)
    h, acc = orc.rkck_control(0.5, 1, 1.0, hmin, hmax)
    assert acc == 0 and h == pytest.approx(0.1)
    # clamp to [hmin, hmax] on acceptance
    h, acc = orc.rkck_control(1e-9, 0, 9.0, hmin, hmax)
    assert h == hmax


# ----------------------------------------------------------------- whole runs
@pytest.mark.parametrize("lam,T", [(-1.0, 3.0), (0.5, 2.0), (-20.0, 1.0)])
def test_adaptive_linear_closed_form(orc, lam, T):
    pb = orc.linear([[lam]])
    rtol = 1e-9
    y1, st, stats = orc.rkck_solve(pb, None, [1.0], 0.0, T, rtol, 0.0)
    assert st == orc.OK
    assert abs(y1[0] - math.exp(lam * T)) <= 100 * rtol * math.exp(lam * T) + 1e-300
    assert stats[orc.ST_ACCEPT] > 0
    assert stats[orc.ST_RHS] == 6 * stats[orc.ST_ACCEPT] + 5 * stats[orc.ST_REJECT]


def test_vdp_accuracy_and_tolerance_proportionality(orc):
    pb = orc.vdp()
    mu, y0 = 1.7, np.array([1.5, -0.2])
    ex = _vdp_exact(y0, mu, 10.0)
    errs = []
    for rtol in (1e-6, 1e-8, 1e-10):
        y1, st, _ = orc.rkck_solve(pb, [mu], y0, 0.0, 10.0, rtol, rtol * 1e-2)
        assert st == orc.OK
        errs.append(np.abs(y1 - ex).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 1e3 * 1e-8


def test_end_point_and_no_op(orc):
    pb = orc.vdp()
    y1, st, stats = orc.rkck_solve(pb, [1.0], [0.3, 0.1], 2.0, 2.0, 1e-8, 1e-10)
    assert st == orc.OK and list(y1) == [0.3, 0.1] and stats[orc.ST_ACCEPT] == 0


def test_guards(orc):
    pb = orc.vdp()
    _, st, stats = orc.rkck_solve(pb, [1.0], [1.0, 0.0], 0.0, 10.0, 1e-8, 1e-10, max_steps=5)
    assert st == orc.MAXSTEPS and stats[0] + stats[1] == 5
    # overflowing linear growth: NaN error estimates shrink h below hMin
    pb = orc.linear([[1e300]])
    _, st, _ = orc.rkck_solve(pb, None, [1.0], 0.0, 1.0, 1e-8, 0.0)
    assert st == orc.HMIN


def test_batch_equals_single(orc):
    from paper_1611_02274_amd import inputs as I
    pb = orc.vdp()
    y0, g = I.vdp_inputs(64, 7)
    y1, status, stats = orc.rkck_batch(pb, y0, g, 0.0, 5.0, 1e-8, 1e-10, n_threads=4)
    for i in (0, 17, 63):
        ys, st, s1 = orc.rkck_solve(pb, g[:, i], y0[:, i], 0.0, 5.0, 1e-8, 1e-10)
        assert np.array_equal(ys, y1[:, i]) and st == status[i]
        assert np.array_equal(s1, stats[:, i])
