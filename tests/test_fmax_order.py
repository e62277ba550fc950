"""The RKCK error maximum does not depend on the order of its fmax operations
(CPU only).

The controller (Sec. 3.1) takes the largest scaled error component.  The
oracle folds t_0 .. t_{N-1} into fmax from 0 in species order; the group
kernels let each lane fold the slots it owns (k = m L + r) from 0 and then
combine the L lane values in a butterfly (lane r with lane r ^ o for
o = 1, 2, 4, ...).  With t_k >= +0 or NaN both give the largest non-NaN value
(0 when every t_k is NaN), bit for bit; this models both orders in numpy and
compares them on inputs with NaNs, zeros, ties and denormals."""
import numpy as np
import pytest


def serial_max(t):
    s = 0.0
    for v in t:
        s = float(np.fmax(s, v))
    return s


def butterfly_max(t, L):
    n = len(t)
    lane = [0.0] * L
    for k in range(n):
        r = k % L
        lane[r] = float(np.fmax(lane[r], t[k]))
    o = 1
    while o < L:
        lane = [float(np.fmax(lane[r], lane[r ^ o])) for r in range(L)]
        o <<= 1
    assert len({np.float64(v).tobytes() for v in lane}) == 1   # every lane agrees
    return lane[0]


def _cases(rng, n):
    yield np.abs(rng.standard_normal(n)) * 10.0 ** rng.integers(-300, 300, n)
    t = np.abs(rng.standard_normal(n))
    t[rng.random(n) < 0.3] = np.nan
    yield t
    yield np.full(n, np.nan)
    yield np.zeros(n)
    t = np.full(n, 2.5)
    t[rng.integers(0, n)] = np.nan
    yield t
    yield np.abs(rng.standard_normal(n)) * 5e-324
    t = np.abs(rng.standard_normal(n))
    t[rng.integers(0, n)] = np.inf
    yield t


@pytest.mark.parametrize("n,L", [(28, 8), (13, 16), (32, 16), (53, 32), (9, 16), (1, 8)])
def test_butterfly_equals_serial(n, L):
    rng = np.random.default_rng(1000 * n + L)
    for _ in range(50):
        for t in _cases(rng, n):
            a, b = serial_max(t), butterfly_max(t, L)
            assert np.float64(a).tobytes() == np.float64(b).tobytes(), (t, a, b)
            finite = t[~np.isnan(t)]
            assert a == (finite.max() if finite.size and finite.max() > 0 else 0.0)
