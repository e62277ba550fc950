"""Correctly rounded exp / log / pow: the oracle's (binary128) and the HIP
kernels' (double-double, evaluated here on the host from the same source the
GPU runs) both equal the exact value rounded to nearest, computed by mpmath."""
import ctypes as C

import mpmath as mp
import numpy as np
import pytest

mp.mp.prec = 240


def _cr(v) -> float:
    return float(v)   # mpf -> nearest double


def _inputs(seed=0, n=4000):
    rng = np.random.default_rng(seed)
    xe = np.concatenate([rng.uniform(-40, 40, n), rng.uniform(-700, 700, n // 4),
                         rng.uniform(-1e-6, 1e-6, n // 8), [0.0, 1e-300, -1e-300, 709.78, -708.0]])
    xl = np.concatenate([rng.uniform(500, 3500, n), 10 ** rng.uniform(-300, 300, n // 2),
                         rng.uniform(0.999, 1.001, n // 8), [1.0, 2.0, 0.5, 1e-310, 5e-324]])
    xp = np.concatenate([rng.uniform(0, 2, n), 10 ** rng.uniform(-30, 10, n // 2),
                         [1e-300, 0.5, 1.0, 7.0, 1e-310]])
    return xe, xl, xp


POW_EXPONENTS = (-0.2, -0.25, 1.0 / 3.0, 2.0 / 3.0)


def _refs(xe, xl, xp):
    re = [_cr(mp.exp(mp.mpf(float(x)))) for x in xe]
    rl = [_cr(mp.log(mp.mpf(float(x)))) for x in xl]
    rp = {y: [_cr(mp.power(mp.mpf(float(x)), mp.mpf(y))) for x in xp] for y in POW_EXPONENTS}
    return re, rl, rp


@pytest.fixture(scope="module")
def refs():
    xe, xl, xp = _inputs()
    return (xe, xl, xp), _refs(xe, xl, xp)


def test_oracle_is_correctly_rounded(orc, refs):
    (xe, xl, xp), (re, rl, rp) = refs
    assert [orc.cr_exp(x) for x in xe] == re
    assert [orc.cr_log(x) for x in xl] == rl
    for y in POW_EXPONENTS:
        assert [orc.cr_pow(x, y) for x in xp] == rp[y]


def test_oracle_special_values(orc):
    inf, nan = float("inf"), float("nan")
    assert orc.cr_exp(1000.0) == inf and orc.cr_exp(-1000.0) == 0.0
    assert np.isnan(orc.cr_exp(nan)) and np.isnan(orc.cr_log(-1.0))
    assert orc.cr_log(0.0) == -inf and orc.cr_log(inf) == inf
    assert orc.cr_pow(0.0, -0.2) == inf and orc.cr_pow(0.0, 1 / 3) == 0.0
    assert orc.cr_pow(inf, -0.25) == 0.0 and orc.cr_pow(inf, 2 / 3) == inf
    assert np.isnan(orc.cr_pow(nan, 1 / 3)) and np.isnan(orc.cr_pow(-2.0, 1 / 3))
    assert orc.cr_pow(1.0, nan) == 1.0 and orc.cr_pow(nan, 0.0) == 1.0


def _kernel_math():
    from paper_1611_02274_amd import _lib
    L = _lib.lib()
    f = L.rkmi_crmath_host
    f.argtypes = [C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
    f.restype = C.c_int

    def run(fn, x, y=None):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(np.zeros_like(x) if y is None else y, dtype=np.float64)
        out = np.zeros_like(x)
        assert f(fn, x.size, x.ctypes.data, y.ctypes.data, out.ctypes.data) == 0
        return out
    return run


def test_kernel_math_is_correctly_rounded(refs):
    (xe, xl, xp), (re, rl, rp) = refs
    run = _kernel_math()
    assert run(0, xe[np.abs(xe) < 708]).tolist() == [r for x, r in zip(xe, re) if abs(x) < 708]
    assert run(1, xl).tolist() == rl
    for y in POW_EXPONENTS:
        assert run(2, xp, np.full(xp.size, y)).tolist() == rp[y]


def test_kernel_math_matches_oracle_bulk(orc):
    """A larger sample against the oracle (both must be the correctly rounded value)."""
    run = _kernel_math()
    rng = np.random.default_rng(7)
    x = rng.uniform(-45, 45, 200_000)
    assert np.array_equal(run(0, x), np.array([orc.cr_exp(v) for v in x]))
    x = rng.uniform(300, 4000, 100_000)
    assert np.array_equal(run(1, x), np.array([orc.cr_log(v) for v in x]))
    x = 10 ** rng.uniform(-20, 3, 200_000)
    for y in POW_EXPONENTS:
        assert np.array_equal(run(2, x, np.full(x.size, y)),
                              np.array([orc.cr_pow(v, y) for v in x]))


def test_kernel_pow_third_is_correctly_rounded(orc):
    """The RKC controllers' x^RN(1/3) and x^RN(2/3) (cube root refined in
    double-double, times x^(RN(1/3) - 1/3); the second power as the square of
    the first) are the correctly rounded powers: errors in [0, 1], rejected
    errors above 1, subnormals, and the exact cases."""
    run = _kernel_math()
    rng = np.random.default_rng(5)
    x = np.concatenate([10 ** rng.uniform(-300, 0, 3000), rng.uniform(0, 1, 3000),
                        1.0 - 10 ** rng.uniform(-16, -3, 500), 1.0 + 10 ** rng.uniform(-16, -1, 300),
                        10 ** rng.uniform(0, 300, 1000), 2.0 ** rng.integers(-1074, 1023, 300),
                        [0.0, 1.0, 5e-324, 2.0 ** -1022, 2.0 ** -1074 * 3, 0.5, 0.999999, 8.0,
                         1.7976931348623157e308]])
    y = np.zeros(x.size)
    p1, p2, p3 = run(3, x, y), run(4, x, y), run(5, x, y)
    assert p1.tolist() == [_cr(mp.power(mp.mpf(float(v)), mp.mpf(1.0 / 3.0))) for v in x]
    assert p2.tolist() == [_cr(mp.power(mp.mpf(float(v)), mp.mpf(2.0 / 3.0))) for v in x]
    assert np.array_equal(p3.view(np.int64), p1.view(np.int64))
    xb = np.concatenate([rng.uniform(0, 1, 150_000), 10 ** rng.uniform(0, 12, 50_000)])
    yb = np.zeros(xb.size)
    assert np.array_equal(run(3, xb, yb), np.array([orc.cr_pow(v, 1.0 / 3.0) for v in xb]))
    assert np.array_equal(run(4, xb, yb), np.array([orc.cr_pow(v, 2.0 / 3.0) for v in xb]))


def test_kernel_rkck_powers_are_correctly_rounded(orc):
    """The RKCK controllers' err^-0.25 (fourth root refined in double-double)
    and err^-RN(0.2) (fifth root times x^-(RN(0.2) - 1/5)) are the correctly
    rounded powers over the whole positive range."""
    run = _kernel_math()
    rng = np.random.default_rng(9)
    x = np.concatenate([10 ** rng.uniform(-300, 300, 4000), rng.uniform(1e-4, 1, 3000),
                        rng.uniform(1, 100, 2000), 1.0 + 10 ** rng.uniform(-16, -2, 300),
                        1.0 - 10 ** rng.uniform(-16, -2, 300), 2.0 ** rng.integers(-1074, 1023, 300),
                        # within a few ulps of 1 the values lie near rounding midpoints
                        1.0 + np.arange(1, 64) * 2.0 ** -52, 1.0 - np.arange(1, 64) * 2.0 ** -53,
                        1.0 + np.arange(1, 64) * 2.0 ** -40,
                        np.outer(16.0 ** np.arange(-20, 20), 1.0 + np.arange(-8, 9) * 2.0 ** -52).ravel(),
                        np.outer(32.0 ** np.arange(-20, 20), 1.0 + np.arange(-8, 9) * 2.0 ** -52).ravel(),
                        [1.0, 5e-324, 2.0 ** -1022, 16.0, 32.0, 0.0625, 1.7976931348623157e308]])
    y = np.zeros(x.size)
    for fn, p in ((6, -0.25), (7, -0.2)):
        got = run(fn, x, y)
        assert got.tolist() == [_cr(mp.power(mp.mpf(float(v)), mp.mpf(p))) for v in x], fn
        xb = np.concatenate([rng.uniform(1e-4, 1, 100_000), 10 ** rng.uniform(0, 10, 50_000)])
        assert np.array_equal(run(fn, xb, np.zeros(xb.size)),
                              np.array([orc.cr_pow(v, p) for v in xb])), fn


def test_kernel_math_special_values():
    run = _kernel_math()
    inf, nan = float("inf"), float("nan")
    e = run(0, [1000.0, -1000.0, nan])
    assert e[0] == inf and e[1] == 0.0 and np.isnan(e[2])
    lg = run(1, [0.0, -1.0, inf, 1.0])
    assert lg[0] == -inf and np.isnan(lg[1]) and lg[2] == inf and lg[3] == 0.0
    p = run(2, [0.0, 0.0, inf, nan, 1.0, -8.0], [-0.2, 1 / 3, -0.25, 0.5, nan, 1 / 3])
    assert p[0] == inf and p[1] == 0.0 and p[2] == 0.0 and np.isnan(p[3]) and p[4] == 1.0
    assert np.isnan(p[5])
