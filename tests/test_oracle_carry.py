"""Pins of the oracle's carried controller state (the alternative to the
restart at every global step that Sec. 3 mentions): a cleared state is exactly
the restart; carried substeps keep the accuracy of the method against an
independent integrator while skipping the restart's first-step selection and
most spectral-radius estimates."""
import numpy as np

from paper_1611_02274_amd import inputs as I


def _substeps(orc, fn, pb, y0, g, T, k, rtol, atol, carry=None):
    y, rhs, acc = y0, 0, 0
    for s in range(k):
        if carry is None:
            y, st, stats = fn(pb, y, g, s * T / k, (s + 1) * T / k, rtol, atol)
        else:
            y, st, stats = fn(pb, y, g, carry, s * T / k, (s + 1) * T / k, rtol, atol)
        assert np.all(st == 0)
        rhs += stats[2].astype(np.int64)
        acc += stats[0].astype(np.int64)
    return y, rhs, acc


def test_cleared_carry_is_the_restart(orc):
    net = I.standard_network(13)
    pb = orc.network(net)
    y0, g = I.kinetics_inputs(net, 40, 12)
    for fn, fc, t1 in ((orc.rkc_batch, orc.rkc_batch_carry, 1e-6),
                       (orc.rkck_batch, orc.rkck_batch_carry, 1e-8)):
        c = orc.carry_init(pb, 40)
        a = fn(pb, y0, g, 0.0, t1, 1e-8, 1e-12)
        b = fc(pb, y0, g, c, 0.0, t1, 1e-8, 1e-12)
        for x, y in zip(a, b):
            assert np.array_equal(np.asarray(x), np.asarray(y))
        assert np.all(c[0] == 1.0) and np.all(c[1] > 0.0)
        # an empty interval leaves a carried state as it is
        c2 = c.copy()
        fc(pb, a[0], g, c2, t1, t1, 1e-8, 1e-12)
        assert np.array_equal(c2, c)


def test_carried_substeps_accuracy_and_work(orc):
    """van der Pol over [0, 4] in 40 substeps: with the state carried, RKC and
    RKCK stay as accurate (against DOP853 at rtol 1e-13) as with restarts and
    use fewer right-hand sides; RKC also runs fewer spectral-radius estimates."""
    from scipy.integrate import solve_ivp
    pb = orc.vdp()
    y0, g = I.vdp_inputs(6, 31)
    ref = np.stack([solve_ivp(lambda t, y: orc.rhs(pb, g[:, i], y), (0.0, 4.0), y0[:, i],
                              method="DOP853", rtol=1e-13, atol=1e-13).y[:, -1]
                    for i in range(6)], 1)
    for fn, fc in ((orc.rkc_batch, orc.rkc_batch_carry), (orc.rkck_batch, orc.rkck_batch_carry)):
        yr, rhs_r, _ = _substeps(orc, fn, pb, y0, g, 4.0, 40, 1e-8, 1e-10)
        c = orc.carry_init(pb, 6)
        yc, rhs_c, _ = _substeps(orc, fc, pb, y0, g, 4.0, 40, 1e-8, 1e-10, carry=c)
        err_r = np.abs(yr - ref).max()
        err_c = np.abs(yc - ref).max()
        assert err_c <= max(3.0 * err_r, 1e-6), (err_r, err_c)
        assert np.all(rhs_c < rhs_r), (rhs_c, rhs_r)


def test_carried_rkc_refreshes_spectral_radius_on_schedule(orc):
    """With the state carried, the accepted-step count runs on across calls, so
    the spectral radius is estimated when it crosses a multiple of 25 and after
    rejections, not at every call's start."""
    net = I.standard_network(13)
    pb = orc.network(net)
    y0, g = I.kinetics_inputs(net, 8, 5)
    c = orc.carry_init(pb, 8)
    y, sr_total, n_acc = y0, 0, 0
    for s in range(10):
        y, st, stats = orc.rkc_batch_carry(pb, y, g, c, s * 1e-7, (s + 1) * 1e-7, 1e-8, 1e-12)
        if s > 0:
            # a call starting between refreshes adds only one estimate per 25
            # accepted steps crossed and one per rejection
            crossed = (c[5] // 25) - ((c[5] - stats[0]) // 25)
            assert np.all(stats[3] <= crossed + stats[1] + 1)
        sr_total += stats[3]
    assert np.all(c[0] == 1.0)
