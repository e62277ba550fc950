"""Roundoff-free pins of the oracle's discrete adjoints: the gradient of
L = w . y(t1) through the replayed step map (step sizes, and RKC stage counts,
held at the recorded values) against complex-step derivatives of that same
replay, Im L(y0 + i e v, theta + i e u) / e, which involve no subtraction of
nearly equal values and so resolve every component of every system to about
1e-13.  Planted mistakes in the adjoint recursions must fail."""
import numpy as np
import pytest

from paper_1611_02274_amd import inputs as I

from .test_oracle_rkc_driver import _mutant


def _cs_gradient(orc, method, pb, g, y0, rec, w):
    """Every component of dL/dy0 and dL/dtheta by complex steps along the unit
    directions."""
    n, nt = pb.n_eq, pb.n_theta
    if method == "rkc":
        hs, ss = rec

        def jvp(dy, dth):
            return orc.rkc_replay_jvp_cs(pb, g, y0, 0.0, hs, ss, w, dy, dth)
    else:
        def jvp(dy, dth):
            return orc.rkck_replay_jvp_cs(pb, g, y0, 0.0, rec, w, dy, dth)
    gy = np.array([jvp(np.eye(n)[m], np.zeros(nt)) for m in range(n)])
    gt = np.array([jvp(np.zeros(n), np.eye(nt)[j]) for j in range(nt)])
    return gy, gt


def _cases():
    net13, net9 = I.standard_network(13), I.standard_network(9)
    out = []
    y0, g = I.vdp_inputs(3, 41)
    for i in range(3):
        out.append(("vdp", y0[:, i], g[:, i], 2.0, 1e-8, 1e-10, 2, None))
    for net, t1, seed in ((net13, 1e-6, 5005), (net9, 3e-7, 43)):
        y0, g = I.kinetics_inputs(net, 3, seed, (1000.0, 2500.0))
        for i in range(3):
            out.append((f"net{net.n_sp}", y0[:, i], g[:, i], t1, 1e-8, 1e-12, net.n_sp, net))
    return out


def _problem(orc, name, net):
    return orc.vdp() if name == "vdp" else orc.network(net)


def check_adjoints(orc, methods=("rkc", "rkck")):
    rng = np.random.default_rng(5)
    for method in methods:
        for name, y0, g, t1, rtol, atol, n, net in _cases():
            pb = _problem(orc, name, net)
            if method == "rkck" and name != "vdp":
                t1 = t1 / 20.0
            w = rng.standard_normal(n)
            if method == "rkc":
                _, st, stats, hs, ss = orc.rkc_solve(pb, g, y0, 0.0, t1, rtol, atol)
                rec = (hs, ss)
                dy, dth = orc.rkc_replay_adjoint(pb, g, y0, 0.0, hs, ss, w)
            else:
                _, st, stats, hs = orc.rkck_solve_rec(pb, g, y0, 0.0, t1, rtol, atol)
                rec = hs
                dy, dth = orc.rkck_replay_adjoint(pb, g, y0, 0.0, hs, w)
            assert st == orc.OK and stats[orc.ST_ACCEPT] >= 3
            gy, gt = _cs_gradient(orc, method, pb, g, y0, rec, w)
            assert np.abs(dy - gy).max() <= 1e-12 * np.abs(gy).max(), (method, name)
            assert np.abs(dth - gt).max() <= 1e-12 * np.abs(gt).max(), (method, name)
            # and one random direction through both arguments at once
            v, u = rng.standard_normal(n), rng.standard_normal(pb.n_theta)
            jv = (orc.rkc_replay_jvp_cs(pb, g, y0, 0.0, rec[0], rec[1], w, v, u) if method == "rkc"
                  else orc.rkck_replay_jvp_cs(pb, g, y0, 0.0, rec, w, v, u))
            scale = np.abs(dy * v).sum() + np.abs(dth * u).sum()
            assert abs(dy @ v + dth @ u - jv) <= 1e-12 * scale, (method, name)


def test_adjoints_equal_complex_step_derivatives(orc):
    check_adjoints(orc)


def test_complex_step_on_a_linear_closed_form(orc):
    """y' = A y: the replayed RKC map is y1 = prod_k P_sk(h_k A) y0, so
    dL/dy0 = (prod_k P_sk(h_k A))^T w, formed here from the stability
    polynomial a_s + b_s T_s(w0 + w1 z) by matrix Chebyshev recurrences."""
    A = np.array([[-3.0, 1.0, 0.0], [0.5, -40.0, 2.0], [0.0, 1.0, -700.0]])
    pb = orc.linear(A)
    y0, w = np.array([1.0, -0.5, 0.25]), np.array([0.3, -1.2, 2.0])
    _, st, _, hs, ss = orc.rkc_solve(pb, None, y0, 0.0, 0.05, 1e-6, 1e-9)
    M = np.eye(3)
    for h, s in zip(hs, ss):
        w0 = 1.0 + (2.0 / 13.0) / s ** 2
        th = np.arccosh(w0)
        Ts, dTs = np.cosh(s * th), s * np.sinh(s * th) / np.sinh(th)
        d2Ts = s * (s * np.cosh(s * th) * np.sinh(th) - np.sinh(s * th) * np.cosh(th)) \
            / np.sinh(th) ** 3
        w1 = dTs / d2Ts
        bs = d2Ts / dTs ** 2
        X = w0 * np.eye(3) + w1 * h * A
        Tm, T = np.eye(3), X.copy()
        for _ in range(2, s + 1):
            Tm, T = T, 2.0 * X @ T - Tm
        M = ((1.0 - bs * Ts) * np.eye(3) + bs * T) @ M
    want = M.T @ w
    got = np.array([orc.rkc_replay_jvp_cs(pb, None, y0, 0.0, hs, ss, w, np.eye(3)[m])
                    for m in range(3)])
    assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()


ADJOINT_MUTANTS = {
    "RKC adjoint: nu_j where mu_j carries wbar_j to wbar_{j-1}": (
        "        wb1[i] += tb.mu[j] * wbj[i];\n", "        wb1[i] += tb.nu[j] * wbj[i];\n"),
    "RKC adjoint: first stage's theta term dropped": (
        "    rhs_vjp(S, Wst, f0b, jtu, th);\n    for (int i = 0; i < N; ++i) lam[i] = Wb[i] + jtu[i];\n"
        "    for (int q = 0; q < NT; ++q) thacc[q] += th[q];\n",
        "    rhs_vjp(S, Wst, f0b, jtu, th);\n    for (int i = 0; i < N; ++i) lam[i] = Wb[i] + jtu[i];\n"),
    "RKCK adjoint: embedded weights c* in place of c": (
        "      for (int i = 0; i < N; ++i) kb[st][i] = RKCK_C[st] * lam[i];",
        "      for (int i = 0; i < N; ++i) kb[st][i] = RKCK_CS[st] * lam[i];"),
}


@pytest.mark.parametrize("name", sorted(ADJOINT_MUTANTS))
def test_planted_adjoint_mistake_is_caught(orc, tmp_path, name):
    old, new = ADJOINT_MUTANTS[name]
    with _mutant(orc, tmp_path, old, new) as m:
        with pytest.raises(AssertionError):
            check_adjoints(m, ("rkck",) if "RKCK" in name else ("rkc",))
