"""Pins of the oracle's Gershgorin spectral-radius bound (the Appendix names
the circle theorem as an alternative to the power method): the analytic
Jacobian against central differences of the right-hand side, the bound
against the infinity norm and the eigenvalues of that finite-difference
Jacobian, and RKC integrations with the bound against those with the power
method (both solve the same equations)."""
import numpy as np
import pytest

from paper_1611_02274_amd import inputs as I


def _fd_jacobian(orc, pb, g, y):
    n = y.size
    J = np.zeros((n, n))
    for i in range(n):
        h = 1e-6 * max(abs(y[i]), 1e-6)
        yp, ym = y.copy(), y.copy()
        yp[i] += h
        ym[i] -= h
        J[:, i] = (orc.rhs(pb, g, yp) - orc.rhs(pb, g, ym)) / (yp[i] - ym[i])
    return J


def _cases(orc, name, n, seed):
    if name == "vdp":
        y0, g = I.vdp_inputs(n, seed, (0.5, 3000.0))
        return orc.vdp(orc.SR_GERSHGORIN), y0, g
    net = I.standard_network(int(name[3:]))
    y0, g = I.kinetics_inputs(net, n, seed, (900.0, 2800.0))
    return orc.network(net, orc.SR_GERSHGORIN), y0, g


@pytest.mark.parametrize("name", ["vdp", "net9", "net13"])
def test_jacobian_matches_central_differences(orc, name):
    pb, y0, g = _cases(orc, name, 12, 41)
    for i in range(y0.shape[1]):
        sig, J = pb.gershgorin(g[:, i], y0[:, i])
        Jfd = _fd_jacobian(orc, pb, g[:, i], y0[:, i].copy())
        scale = np.abs(J).max()
        assert np.abs(J - Jfd).max() <= 1e-6 * scale, (name, i)


@pytest.mark.parametrize("name", ["vdp", "net9", "net13"])
def test_bound_is_the_row_norm_and_bounds_the_eigenvalues(orc, name):
    pb, y0, g = _cases(orc, name, 12, 43)
    for i in range(y0.shape[1]):
        sig, _ = pb.gershgorin(g[:, i], y0[:, i])
        Jfd = _fd_jacobian(orc, pb, g[:, i], y0[:, i].copy())
        assert sig == pytest.approx(np.linalg.norm(Jfd, np.inf), rel=1e-6)
        assert sig >= np.abs(np.linalg.eigvals(Jfd)).max() * (1 - 1e-6)


def test_vdp_bound_special_values(orc):
    """At y = 0 the van der Pol Jacobian is [[0, 1], [-1, mu]]: bound 1 + mu."""
    pb = orc.vdp(orc.SR_GERSHGORIN)
    for mu in (0.5, 7.0, 3000.0):
        sig, J = pb.gershgorin(np.array([mu]), np.zeros(2))
        assert sig == 1.0 + mu
        assert np.array_equal(J, np.array([[0.0, 1.0], [-1.0, mu]]))


@pytest.mark.parametrize("name,t1,rtol,atol", [("vdp", 1.0, 1e-6, 1e-8),
                                               ("net13", 1e-6, 1e-8, 1e-12)])
def test_rkc_with_the_bound_solves_the_same_problem(orc, name, t1, rtol, atol):
    pb, y0, g = _cases(orc, name, 24, 45)
    pp = orc.vdp() if name == "vdp" else orc.network(pb.net)
    yg, sg, stg = orc.rkc_batch(pb, y0, g, 0.0, t1, rtol, atol)
    yp, sp, stp = orc.rkc_batch(pp, y0, g, 0.0, t1, rtol, atol)
    assert np.all(sg == 0) and np.all(sp == 0)
    scale = np.abs(yp).max(axis=0) + atol / rtol
    assert np.all(np.abs(yg - yp).max(axis=0) <= 1e3 * rtol * scale)
    assert np.all(stg[4] == 0)                  # no power-method iterations
    assert np.all(stg[3] >= 1)                  # the bound was formed


def test_option_rejected_where_no_jacobian(orc):
    pb = orc.pleiades()
    pb.s.sr_method = 1
    y0, _ = I.pleiades_inputs(2, 6006)
    with pytest.raises(Exception):
        orc.rkc_batch(pb, y0, None, 0.0, 0.1, 1e-8, 1e-10)
