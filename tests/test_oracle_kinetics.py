"""Pins of the oracle's mass-action right-hand side (Sec. 4.2 species equations,
Arrhenius rate coefficients) against conservation laws, closed-form solutions of
single-reaction systems, special cases of the Arrhenius law, chemical
equilibrium and finite differences."""
import math
from dataclasses import replace

import numpy as np
import pytest

from paper_1611_02274_amd import inputs as I


@pytest.mark.parametrize("n_sp", [9, 13, 32, 53])
def test_generator_balanced_and_deterministic(n_sp):
    net = I.standard_network(n_sp)
    nu = net.stoich()
    assert net.n_rx == I.NETWORK_SIZES[n_sp]
    assert np.all(net.W @ nu == 0)              # mass balance
    assert np.all(net.comp.T @ nu == 0)         # element balance
    used = set(net.reac[net.reac >= 0]) | set(net.prod[net.prod >= 0])
    assert used == set(range(n_sp))
    assert len({tuple(c) for c in net.comp}) == n_sp
    net2 = I.standard_network(n_sp)
    assert np.array_equal(net.reac, net2.reac) and np.array_equal(net.lnA, net2.lnA)


def test_inputs_shapes_and_ranges():
    net = I.standard_network(13)
    y0, g = I.kinetics_inputs(net, 1000, 5)
    assert y0.shape == (13, 1000) and g.shape == (2, 1000)
    assert np.allclose(y0.sum(0), 1.0, atol=1e-14) and np.all(y0 > 0)
    assert np.all((g[0] >= 1000) & (g[0] <= 2500)) and np.all(g[1] > 0)
    y0v, gv = I.vdp_inputs(4096, 1)
    assert y0v.shape == (2, 4096) and gv.shape == (1, 4096)
    assert np.all(np.abs(y0v) <= 2) and np.all((gv >= 0.5) & (gv <= 2))


def _net_one(reac, prod, W, lnA=0.0, beta=0.0, Ea=0.0, K=1e300):
    comp = np.array([[int(w), 0, 0] for w in W])
    return I.Network(n_sp=len(W), n_rx=1, comp=comp, W=np.array(W, dtype=float),
                     reac=np.array([reac], dtype=np.int32),
                     prod=np.array([prod], dtype=np.int32),
                     lnA=np.array([lnA]), beta=np.array([beta]), Ea=np.array([Ea]),
                     Keq=np.array([K]))


@pytest.mark.parametrize("n_sp", [13, 53])
def test_rhs_conserves_mass_and_elements(orc, n_sp):
    net = I.standard_network(n_sp)
    pb = orc.network(net)
    y0, g = I.kinetics_inputs(net, 8, 99)
    for i in range(8):
        f = orc.rhs(pb, g[:, i], y0[:, i])
        scale = np.abs(f).sum()
        assert scale > 0
        assert abs(f.sum()) <= 1e-13 * scale
        elem = net.comp.T @ (f / net.W)
        assert np.all(np.abs(elem) <= 1e-13 * np.abs(f / net.W).sum())


def test_dimerisation_closed_form(orc):
    """A + A -> A2 with negligible reverse rate and k = A (beta = Ea = 0):
    dC_A/dt = -2 k C_A^2, so C_A(t) = C_A0 / (1 + 2 k C_A0 t)."""
    k, rho = 3.0e9, 2.0e-4
    net = _net_one([0, 0], [1, -1], [1.0, 2.0], lnA=math.log(k))
    pb = orc.network(net)
    Y0 = np.array([0.6, 0.4])
    T = 1.0e-5 * 1.0 / (2 * k * rho * 0.6)   # about the half-life scale
    t1 = 5 * T / 1e-5
    y1, st, _ = orc.rkck_solve(pb, [1500.0, rho], Y0, 0.0, t1, 1e-11, 1e-15)
    assert st == orc.OK
    CA0 = rho * Y0[0] / 1.0
    CA = CA0 / (1 + 2 * k * CA0 * t1)
    assert y1[0] == pytest.approx(CA * 1.0 / rho, rel=1e-8)
    assert y1[0] + y1[1] == pytest.approx(1.0, rel=1e-13)
    assert y1[0] < 0.5 * Y0[0]


def test_third_body_decomposition_closed_form(orc):
    """A2 + M -> A + A (one-species side times [M]) with negligible reverse:
    with x = C_A2 and rho = C_A + 2 x fixed, [M] = rho - x and
    x(t) = rho x0 exp(-k rho t) / (x0 exp(-k rho t) + rho - x0)."""
    k, rho = 2.0e10, 1.5e-4
    net = _net_one([1, -1], [0, 0], [1.0, 2.0], lnA=math.log(k))
    pb = orc.network(net)
    Y0 = np.array([0.3, 0.7])
    t1 = 1.0 / (k * rho)
    y1, st, _ = orc.rkck_solve(pb, [1200.0, rho], Y0, 0.0, t1, 1e-11, 1e-15)
    assert st == orc.OK
    x0 = rho * Y0[1] / 2.0
    e = math.exp(-k * rho * t1)
    x = rho * x0 * e / (x0 * e + rho - x0)
    assert y1[1] == pytest.approx(x * 2.0 / rho, rel=1e-8)


def test_arrhenius_special_cases(orc):
    Y, rho = np.array([0.5, 0.5]), 1e-4

    def rate(T, **kw):
        pb = orc.network(_net_one([0, 0], [1, -1], [1.0, 2.0], **kw))
        return orc.rhs(pb, [T, rho], Y)[1]

    # b = 1, E = 0: k proportional to T
    assert rate(2000.0, beta=1.0) / rate(1000.0, beta=1.0) == pytest.approx(2.0, rel=1e-13)
    # b = 1/2: k(4T) / k(T) = 2
    assert rate(4000.0, beta=0.5) / rate(1000.0, beta=0.5) == pytest.approx(2.0, rel=1e-13)
    # b = 0, E = 1000 K: k(500) / k(1000) = exp(-2) / exp(-1)
    assert rate(500.0, Ea=1000.0) / rate(1000.0, Ea=1000.0) == pytest.approx(math.exp(-1),
                                                                             rel=1e-13)
    # ln A shifts the rate by a factor
    assert rate(1000.0, lnA=math.log(2.0)) / rate(1000.0) == pytest.approx(2.0, rel=1e-13)


def test_equilibrium_gives_zero_rate(orc):
    """A + A <=> A2 (+M on the dimer side): net rate zero when
    C_A^2 / (C_A2 [M]) = k_r / k_f = 1 / K."""
    K, W = 1.0e7, [1.0, 2.0]
    net = _net_one([0, 0], [1, -1], W, lnA=math.log(1e11), K=K)
    pb = orc.network(net)
    CA = 2.0e-6
    # C_B (C_A + C_B) = K C_A^2
    CB = (-CA + math.sqrt(CA * CA + 4 * K * CA * CA)) / 2
    rho = CA * W[0] + CB * W[1]
    Y = np.array([CA * W[0] / rho, CB * W[1] / rho])
    f = orc.rhs(pb, [1000.0, rho], Y)
    flux = 1e11 * CA * CA * 2 / rho
    assert np.all(np.abs(f) <= 1e-12 * flux)
    # and integrating from there stays there
    y1, st, _ = orc.rkck_solve(pb, [1000.0, rho], Y, 0.0, 1e-6, 1e-10, 1e-16)
    assert np.allclose(y1, Y, rtol=1e-10)


@pytest.mark.parametrize("n_sp", [9, 13])
def test_vjp_matches_finite_differences(orc, n_sp):
    net = I.standard_network(n_sp)
    pb = orc.network(net)
    y0, g = I.kinetics_inputs(net, 3, 17)
    rng = np.random.default_rng(4)
    for i in range(3):
        y, gi = y0[:, i], g[:, i]
        u = rng.standard_normal(n_sp)
        jtu, dth = orc.rhs_vjp(pb, gi, y, u)
        # f is quadratic in y (bimolecular rate laws), so a central difference is
        # exact for any step: a large step keeps round-off out of the comparison
        for m in range(n_sp):
            e = 1e-2 * y[m]
            yp, ym = y.copy(), y.copy()
            yp[m] += e
            ym[m] -= e
            fd = (u @ orc.rhs(pb, gi, yp) - u @ orc.rhs(pb, gi, ym)) / (2 * e)
            assert jtu[m] == pytest.approx(fd, rel=1e-9, abs=1e-11 * np.abs(jtu).max())
        for j in range(net.n_rx):
            d = np.zeros(net.n_rx)
            d[j] = 1e-6
            fp = orc.rhs(pb.with_lnA(net.lnA + d), gi, y)
            fm = orc.rhs(pb.with_lnA(net.lnA - d), gi, y)
            fd = (u @ fp - u @ fm) / 2e-6
            assert dth[j] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(dth).max())


def test_vdp_vjp(orc):
    pb = orc.vdp()
    y, u, mu = np.array([0.7, -1.2]), np.array([0.3, 2.0]), 1.4
    jtu, dth = orc.rhs_vjp(pb, [mu], y, u)
    # J = [[0, 1], [-2 mu y1 y2 - 1, mu (1 - y1^2)]]
    J = np.array([[0.0, 1.0], [-2 * mu * y[0] * y[1] - 1, mu * (1 - y[0] ** 2)]])
    assert np.allclose(jtu, J.T @ u, rtol=1e-15)
    assert dth[0] == pytest.approx(u[1] * (1 - y[0] ** 2) * y[1], rel=1e-15)


def test_integrated_invariants_net13(orc):
    net = I.standard_network(13)
    pb = orc.network(net)
    y0, g = I.kinetics_inputs(net, 16, 2002)
    y1, status, stats = orc.rkc_batch(pb, y0, g, 0.0, 1e-6, 1e-8, 1e-12)
    assert np.all(status == orc.OK)
    steps = stats[orc.ST_ACCEPT].max()
    assert np.abs(y1.sum(0) - 1.0).max() <= 1e-15 * steps + 1e-14
    Z0 = net.comp.T @ (y0 / net.W[:, None])
    Z1 = net.comp.T @ (y1 / net.W[:, None])
    assert np.abs(Z1 - Z0).max() <= (1e-15 * steps + 1e-14) * np.abs(Z0).max()
