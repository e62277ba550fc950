"""Pins of the oracle's Pleiades right-hand side (Sec. 4.1) and of RKCK on it:
Newton's third law (momentum and angular momentum balance), the inverse-square
law with the other body's mass, energy conservation along the integration, and
agreement with an independent high-order integrator."""
import numpy as np
import pytest

from paper_1611_02274_amd import inputs as I

M = np.arange(1, 8, dtype=float)


def _acc(orc, s):
    f = orc.rhs(orc.pleiades(), None, s)
    assert np.array_equal(f[:14], s[14:])          # positions' derivatives are the velocities
    return f[14:21], f[21:]


def test_momentum_and_angular_momentum_balance(orc):
    rng = np.random.default_rng(3)
    for _ in range(20):
        s = rng.uniform(-4.0, 4.0, 28)
        ax, ay = _acc(orc, s)
        x, y = s[:7], s[7:14]
        scale = np.abs(M * ax).sum() + np.abs(M * ay).sum()
        assert abs((M * ax).sum()) <= 1e-13 * scale
        assert abs((M * ay).sum()) <= 1e-13 * scale
        torque = (M * (x * ay - y * ax)).sum()
        assert abs(torque) <= 1e-13 * np.abs(M * (x * ay - y * ax)).sum() * 10


@pytest.mark.parametrize("k,j", [(0, 6), (3, 1), (6, 2)])
def test_inverse_square_with_other_mass(orc, k, j):
    """Body k at the origin, body j at distance d along a direction, the rest
    10^8 away: k's acceleration is m_j / d^2 towards j (m_j = j + 1)."""
    d, th = 1.7, 0.6
    s = np.zeros(28)
    far = [i for i in range(7) if i not in (k, j)]
    for n_, i in enumerate(far):
        s[i], s[7 + i] = 1e8 * np.cos(1.0 + n_), 1e8 * np.sin(1.0 + n_)
    s[j], s[7 + j] = d * np.cos(th), d * np.sin(th)
    ax, ay = _acc(orc, s)
    a = M[j] / d ** 2
    assert ax[k] == pytest.approx(a * np.cos(th), rel=1e-12)
    assert ay[k] == pytest.approx(a * np.sin(th), rel=1e-12)
    # and j is pulled back towards k with m_k / d^2
    assert ax[j] == pytest.approx(-M[k] / d ** 2 * np.cos(th), rel=1e-12)


def _energy(s):
    x, y, vx, vy = s[:7], s[7:14], s[14:21], s[21:]
    e = 0.5 * (M * (vx ** 2 + vy ** 2)).sum()
    for i in range(7):
        for j in range(i + 1, 7):
            e -= M[i] * M[j] / np.hypot(x[i] - x[j], y[i] - y[j])
    return e


def test_rkck_conserves_energy_and_matches_dop853(orc):
    """RKCK at eps = 1e-10 over the ten global steps of [0, 1] (each a restart):
    energy drifts by < 1e-8 relative, and the state agrees with scipy's DOP853
    (rtol 1e-13) to 1e-6."""
    from scipy.integrate import solve_ivp
    pb = orc.pleiades()
    y0, _ = I.pleiades_inputs(3, 6006)
    for c in range(3):
        s = y0[:, c].copy()
        e0 = _energy(s)
        for k in range(10):
            s, st, stats = orc.rkck_solve(pb, None, s, 0.1 * k, 0.1 * (k + 1), 1e-10, 0.0)
            assert st == orc.OK and stats[0] > 0
        assert abs(_energy(s) - e0) <= 1e-8 * abs(e0)

        def f(t, z):
            return orc.rhs(pb, None, z)
        ref = solve_ivp(f, (0.0, 1.0), y0[:, c], method="DOP853", rtol=1e-13, atol=1e-13)
        assert np.abs(s - ref.y[:, -1]).max() <= 1e-6 * np.abs(ref.y[:, -1]).max()
