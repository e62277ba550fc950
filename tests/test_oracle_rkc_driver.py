"""Pins of the oracle's RKC driver control flow (Sec. 2.2, driver of Sec. 3.2):
the initial step size, the refresh schedule of the spectral radius, the
stretch of the step to the end point and the step-size sequence, each checked
on a per-attempt trace against values this file computes from the equations
(independent numpy arithmetic), and planted mistakes in the oracle's source
that each of these checks must catch."""
import contextlib
import os
import subprocess

import numpy as np
import pytest

from paper_1611_02274_amd import inputs as I

UROUND = 2.22e-16


def _hmin(t0, t1):
    return 10.0 * UROUND * max(abs(t0), abs(t1 - t0))


# ------------------------------------------------------------ initial step
def _initial_step(f, y0, sigma, t0, t1, rtol, atol):
    """Sec. 2.2: dt0 = 1/sigma (hMax if sigma hMax <= 1, at least hMin),
    Delta_0 = dt0 (f(y0 + dt0 f(y0)) - f(y0)) measured by Eq. E:rmsE with
    weights atol + rtol |y0|, dt1 = 0.1 dt0 / ||Delta_0||^(1/2) within
    [hMin, hMax]."""
    hmax, hmin = t1 - t0, _hmin(t0, t1)
    dt0 = 1.0 / sigma if sigma * hmax > 1.0 else hmax
    dt0 = max(dt0, hmin)
    f0 = f(y0)
    delta0 = dt0 * (f(y0 + dt0 * f0) - f0)
    err0 = np.sqrt(np.mean((delta0 / (atol + rtol * np.abs(y0))) ** 2))
    dt1 = 0.1 * dt0 / np.sqrt(err0) if err0 > 0 else np.inf
    return min(max(dt1, hmin), hmax)


LINEAR_CASES = [
    # (eigenvalues, y0, t1, rtol, atol): sigma hMax > 1, < 1, the hMax clamp
    ([-1.0e3], [1.0], 1.0, 1e-6, 1e-8),
    ([-0.1], [1.0], 1.0, 1e-6, 1e-6),
    ([-1.0e-6], [1.0], 1.0, 1e-3, 1e-3),
    ([-1.0, -50.0, -3.0e3], [1.0, 0.5, -0.2], 2.0, 1e-8, 1e-10),
    ([-4.0, -2.0e5], [0.3, 2.0], 0.5, 1e-5, 1e-9),
]


def check_initial_step(orc):
    for lam, y0, t1, rtol, atol in LINEAR_CASES:
        lam, y0 = np.array(lam), np.array(y0)
        pb = orc.linear(np.diag(lam))
        _, st, _, tr = orc.rkc_trace(pb, None, y0, 0.0, t1, rtol, atol, max_steps=50)
        a = tr[0]
        # sigma of the power method on a linear problem: 1.2 |lambda|_max
        assert abs(a["sigma"] - 1.2 * np.abs(lam).max()) <= 0.012 * 1.2 * np.abs(lam).max()
        want = _initial_step(lambda y: lam * y, y0, a["sigma"], 0.0, t1, rtol, atol)
        m = 1 + int(np.sqrt(1.54 * want * a["sigma"] + 1.0))
        assert a["m"] == m and m < orc.rkc_mmax(rtol)
        assert a["h"] == pytest.approx(want, rel=1e-13, abs=0.0), (lam, y0)
    # van der Pol: f evaluated here, sigma taken from the trace (pinned by the
    # power-method tests)
    for mu, y0, t1 in [(1.0, [2.0, 0.0], 2.0), (30.0, [1.5, -0.5], 1.0), (0.7, [-1.0, 1.3], 0.3)]:
        y0 = np.array(y0)

        def f(y):
            return np.array([y[1], mu * (1.0 - y[0] * y[0]) * y[1] - y[0]])

        _, _, _, tr = orc.rkc_trace(orc.vdp(), [mu], y0, 0.0, t1, 1e-7, 1e-9, max_steps=5)
        want = _initial_step(f, y0, tr[0]["sigma"], 0.0, t1, 1e-7, 1e-9)
        assert tr[0]["h"] == pytest.approx(want, rel=1e-12, abs=0.0), mu


def test_initial_step(orc):
    check_initial_step(orc)


# -------------------------------------------------- spectral radius refresh
def _refresh_runs(orc):
    """Integrations with rejections, some at accepted-step counts that are
    multiples of 25 (where a rejection refreshes sigma twice)."""
    runs = []
    y0, g = I.vdp_inputs(24, 77)
    for i in range(24):
        mu = 5.0 + 40.0 * g[0, i]
        runs.append(orc.rkc_trace(orc.vdp(), [mu], y0[:, i], 0.0, 30.0, 1e-4, 1e-6))
    net = I.standard_network(9)
    y0, g = I.kinetics_inputs(net, 8, 91, (1500.0, 2500.0))
    for i in range(8):
        runs.append(orc.rkc_trace(orc.network(net), g[:, i], y0[:, i], 0.0, 1e-6, 1e-8, 1e-12))
    return runs


def check_refresh(orc, runs):
    n_rej = n_double = 0
    for _, st, stats, tr in runs:
        assert st == orc.OK
        count = 0
        for a in tr:
            if a["nstep"] % 25 == 0:          # the first step and every 25 accepted
                count += 1
            assert a["n_sr"] == count
            if not a["accepted"]:             # and after every rejection
                count += 1
                n_rej += 1
                n_double += a["nstep"] % 25 == 0
        assert stats[orc.ST_SR_CALLS] == count
        assert stats[orc.ST_ACCEPT] == tr["accepted"].sum()
        assert stats[orc.ST_REJECT] == (1 - tr["accepted"]).sum()
    return n_rej, n_double


def test_sigma_refresh_schedule(orc):
    n_rej, n_double = check_refresh(orc, _refresh_runs(orc))
    # the sample exercises both kinds of refresh after a rejection
    assert n_rej >= 20 and n_double >= 1, (n_rej, n_double)


# ------------------------------------------- step sequence and end stretch
def check_steps(orc, runs, t1_of):
    """Every attempt's proposed step follows from the previous attempt by
    Eq. dtnp1 (accepted: min(10, max(0.1, f)) h with f = 0.8 / err^(1/3) on the
    first accepted step, else 0.8 (h / h_prev) err_prev^(1/3) / err^(2/3);
    rejected: 0.8 h / err^(1/3)) held within [hMin, hMax]; the step taken is
    the time left when that is at most 1.1 times the proposal.  Returns how
    many attempts fell in the window where only the 10% stretch reaches t1."""
    window = 0
    for r, (_, st, _, tr) in enumerate(runs):
        t1 = t1_of(r)
        hmax, hmin = t1, _hmin(0.0, t1)
        prev = None
        for k, a in enumerate(tr):
            left = t1 - a["t"]
            if k > 0:
                b = tr[k - 1]
                if b["accepted"]:
                    if prev is None:
                        fac = min(10.0, 0.8 / b["err"] ** (1.0 / 3.0))
                    else:
                        fac = min(10.0, 0.8 * (b["h"] / prev["h"]) * prev["err"] ** (1.0 / 3.0)
                                  / b["err"] ** (2.0 / 3.0))
                    want = min(max(b["h"] * max(0.1, fac), hmin), hmax)
                    prev = b
                else:
                    want = 0.8 * b["h"] / b["err"] ** (1.0 / 3.0)
                assert a["h_want"] == pytest.approx(want, rel=1e-13, abs=0.0), (r, k)
                expect = left if 1.1 * a["h_want"] >= left else a["h_want"]
                if a["m"] < orc.rkc_mmax(1e-4):   # no stage cap shortened the step
                    assert a["h"] == expect, (r, k)
                window += a["h_want"] < left <= 1.1 * a["h_want"]
            assert a["h"] <= left
        assert st != orc.OK or (tr[-1]["accepted"] and tr[-1]["t"] + tr[-1]["h"] >= t1)
    return window


def _step_runs(orc):
    runs, t1s = [], []
    y0, g = I.vdp_inputs(300, 78)
    for i in range(300):
        t1 = 0.05 + 1.5 * g[0, i]
        runs.append(orc.rkc_trace(orc.vdp(), [1.0 + g[0, i]], y0[:, i], 0.0, t1, 1e-4, 1e-6))
        t1s.append(t1)
    return runs, t1s


def test_step_sequence_and_end_stretch(orc):
    runs, t1s = _step_runs(orc)
    window = check_steps(orc, runs, lambda r: t1s[r])
    assert window >= 5, window


# --------------------------------------------------------- planted mistakes
@contextlib.contextmanager
def _mutant(orc, tmp_path, old, new):
    """The oracle rebuilt from its source with `old` replaced by `new` (which
    must occur once), loaded in place of the real one for the duration."""
    from oracle import build as B
    src = open(B.SRC).read()
    assert src.count(old) == 1, old
    path = os.path.join(str(tmp_path), "rk_oracle_mut.c")
    with open(path, "w") as fh:
        fh.write(src.replace(old, new))
    lib = os.path.join(str(tmp_path), "liborc_mut.so")
    subprocess.run(["gcc", *B.CFLAGS, "-I", os.path.dirname(B.SRC), path, "-o", lib,
                    "-lquadmath", "-lm"], check=True)
    saved_lib, saved_path = orc._lib, B.LIB
    orc._lib, B.LIB = None, lib
    try:
        orc.lib()
        yield orc
    finally:
        orc._lib, B.LIB = saved_lib, saved_path


MUTANTS = {
    "first step without the square root": (
        "return fmax(P1 * dt0 / sqrt(err0), hmin);", "return fmax(P1 * dt0 / err0, hmin);"),
    "first step without the hMax bound on dt0": (
        "if (sigma * dt0 > 1.0) dt0 = 1.0 / sigma;", "dt0 = 1.0 / sigma;"),
    "first-step weights at the tentative state": (
        "w[i] = atol + rtol * fabs(y0[i]);", "w[i] = atol + rtol * fabs(z[i]);"),
    "no sigma refresh after a rejection": (
        "      sigma = rkc_sigma(S, t, y_n, F_n, hmax, v, &n_sr, &n_pow, &n_rhs);\n"
        "      if (!(h >= hmin)) {",
        "      if (!(h >= hmin)) {"),
    "refresh every 25 attempts instead of accepted steps": (
        "if (nstep % SR_PERIOD == 0)", "if (attempts % SR_PERIOD == 0)"),
    "end-point stretch at 1.0": (
        "return (1.1 * h >= fabs(t1 - t)) ? fabs(t1 - t) : h;",
        "return (1.0 * h >= fabs(t1 - t)) ? fabs(t1 - t) : h;"),
    "rejection step with the 2/3 power": (
        "return isfinite(err) ? 0.8 * h / orc_cr_pow(err, 1.0 / 3.0) : P1 * h;",
        "return isfinite(err) ? 0.8 * h / orc_cr_pow(err, 2.0 / 3.0) : P1 * h;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(orc, tmp_path, name):
    old, new = MUTANTS[name]
    with _mutant(orc, tmp_path, old, new) as m:
        caught = []
        for check in (lambda: check_initial_step(m),
                      lambda: check_refresh(m, _refresh_runs(m)),
                      lambda: check_steps(m, *(lambda r: (r[0], lambda i: r[1][i]))(
                          _step_runs(m)))):
            try:
                check()
            except AssertionError:
                caught.append(True)
        assert caught, f"no pin catches: {name}"
