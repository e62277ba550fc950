"""The kernels' per-system code, compiled for the host from the same source as
the GPU kernels, reproduces the oracle bit for bit (CPU only: no GPU used).

This checks the arithmetic of the HIP path (operation order, correctly rounded
transcendentals, controller logic) without a device; the GPU parity tests then
check that the device computes what the host build computes."""
import ctypes as C

import numpy as np
import pytest

from paper_1611_02274_amd import inputs as I


def _host_run(prob, method, y0, g, t0, t1, rtol, atol, max_steps=0):
    from paper_1611_02274_amd import _lib
    f = _lib.lib().rkmi_test_host_integrate
    f.argtypes = [C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                  C.c_double, C.c_double, C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                  C.c_int64]
    f.restype = C.c_int
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    g = np.ascontiguousarray(g if g is not None else np.zeros((1, 1)), dtype=np.float64)
    n = y0.shape[1]
    y1 = np.zeros_like(y0)
    st = np.zeros(n, dtype=np.int32)
    stats = np.zeros((6, n), dtype=np.int32)
    rc = f(0 if method == "rkck" else 1, prob.handle, n, y0.ctypes.data, y1.ctypes.data,
           g.ctypes.data, t0, t1, rtol, atol, st.ctypes.data, stats.ctypes.data, max_steps)
    assert rc == 0
    return y1, st, stats


CASES = [
    ("rkck", "vdp", 200, 1, 0.0, 10.0, 1e-8, 1e-10, None),
    ("rkc", "vdp", 120, 3, 0.0, 2.0, 1e-8, 1e-10, None),
    # stiff: steps of up to and beyond 32 stages (tabulated and formed coefficients)
    ("rkc", "vdp_stiff", 48, 13, 0.0, 1.0, 1e-6, 1e-8, None),
    ("rkc", "net9", 96, 77, 0.0, 1e-6, 1e-8, 1e-12, (800.0, 3000.0)),
    ("rkc", "net13", 96, 2002, 0.0, 1e-6, 1e-8, 1e-12, (1000.0, 2500.0)),
    ("rkck", "net13", 32, 12, 0.0, 2e-8, 1e-8, 1e-12, (1000.0, 2500.0)),
    ("rkck", "net9", 32, 5, 0.0, 1e-8, 1e-6, 0.0, (800.0, 3000.0)),
    # larger networks: vectors and rate constants in slot columns
    ("rkc", "net32", 12, 3003, 0.0, 1e-6, 1e-8, 1e-12, (900.0, 2800.0)),
    ("rkc", "net53", 12, 3003, 0.0, 1e-6, 1e-8, 1e-12, (900.0, 2800.0)),
    ("rkck", "net32", 8, 31, 0.0, 2e-7, 1e-8, 1e-12, (900.0, 2800.0)),
    ("rkck", "net53", 8, 3003, 0.0, 2e-7, 1e-8, 1e-12, (900.0, 2800.0)),
    # networks with the energy equation (state T, Y)
    ("rkc", "net13_thermal", 48, 8008, 0.0, 1e-6, 1e-8, 1e-12, (1000.0, 2500.0)),
    ("rkc", "net9_thermal", 48, 8009, 0.0, 1e-6, 1e-8, 1e-12, (1000.0, 2500.0)),
    ("rkck", "net13_thermal", 16, 8010, 0.0, 5e-8, 1e-8, 1e-12, (1000.0, 2500.0)),
    # the Pleiades problem (28 unknowns in slot columns), one global step
    ("rkck", "pleiades", 24, 6006, 0.0, 0.1, 1e-10, 0.0, None),
    ("rkck", "pleiades", 8, 6007, 0.5, 0.6, 1e-12, 1e-14, None),
    ("rkc", "pleiades", 8, 6008, 0.0, 0.1, 1e-8, 1e-10, None),
]


@pytest.mark.parametrize("method,problem,n,seed,t0,t1,rtol,atol,T_range", CASES)
def test_host_build_of_kernels_equals_oracle(orc, method, problem, n, seed, t0, t1, rtol, atol,
                                             T_range):
    import paper_1611_02274_amd as rk
    if problem in ("vdp", "vdp_stiff"):
        y0, g = I.vdp_inputs(n, seed, (300.0, 3000.0) if problem == "vdp_stiff" else (0.5, 2.0))
        prob, pb = rk.Problem.vdp(), orc.vdp()
    elif problem == "pleiades":
        y0, g = I.pleiades_inputs(n, seed)
        prob, pb = rk.Problem.pleiades(), orc.pleiades()
    elif problem.endswith("_thermal"):
        net = I.thermal_network(int(problem[3:-8]))
        y0, g = I.thermal_inputs(net, n, seed, T_range)
        prob, pb = rk.Problem.network_thermal(net), orc.network_thermal(net)
    else:
        net = I.network_of(problem)
        y0, g = I.kinetics_inputs(net, n, seed, T_range)
        prob, pb = rk.Problem.network(net), orc.network(net)
    yh, sh, sth = _host_run(prob, method, y0, g, t0, t1, rtol, atol)
    fn = orc.rkck_batch if method == "rkck" else orc.rkc_batch
    yo, so, sto = fn(pb, y0, g, t0, t1, rtol, atol)
    assert np.array_equal(sh, so)
    assert np.array_equal(sth, sto), np.argwhere(sth != sto)[:5]
    assert np.array_equal(yh.view(np.int64), yo.view(np.int64))
    if problem == "vdp_stiff":
        assert sto[5].min() <= 32 < sto[5].max()


@pytest.mark.parametrize("problem,n,seed,t1,rtol,atol", [
    ("vdp", 64, 13, 1.0, 1e-6, 1e-8), ("vdp_stiff", 32, 14, 1.0, 1e-6, 1e-8),
    ("net9", 48, 77, 1e-6, 1e-8, 1e-12), ("net13", 48, 2002, 1e-6, 1e-8, 1e-12)])
def test_host_build_gershgorin_equals_oracle(orc, problem, n, seed, t1, rtol, atol):
    """RKC with the Gershgorin bound in place of the power method: the host
    build of the kernels equals the oracle bit for bit."""
    import paper_1611_02274_amd as rk
    from paper_1611_02274_amd import _lib
    if problem.startswith("vdp"):
        y0, g = I.vdp_inputs(n, seed, (300.0, 3000.0) if problem == "vdp_stiff" else (0.5, 2.0))
        prob, pb = rk.Problem.vdp(), orc.vdp(orc.SR_GERSHGORIN)
    else:
        net = I.network_of(problem)
        y0, g = I.kinetics_inputs(net, n, seed, (900.0, 2800.0))
        prob, pb = rk.Problem.network(net), orc.network(net, orc.SR_GERSHGORIN)
    f = _lib.lib().rkmi_test_host_integrate_sr
    f.argtypes = [C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                  C.c_double, C.c_double, C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                  C.c_int64, C.c_int32]
    f.restype = C.c_int
    y0 = np.ascontiguousarray(y0)
    g = np.ascontiguousarray(g)
    yh = np.zeros_like(y0)
    sh = np.zeros(n, dtype=np.int32)
    sth = np.zeros((6, n), dtype=np.int32)
    assert f(1, prob.handle, n, y0.ctypes.data, yh.ctypes.data, g.ctypes.data, 0.0, t1, rtol,
             atol, sh.ctypes.data, sth.ctypes.data, 0, 1) == 0
    yo, so, sto = orc.rkc_batch(pb, y0, g, 0.0, t1, rtol, atol)
    assert np.array_equal(sh, so)
    assert np.array_equal(sth, sto)
    assert np.array_equal(yh.view(np.int64), yo.view(np.int64))
    assert np.all(sto[4] == 0) and np.all(sto[3] >= 1)


def test_host_build_max_steps(orc):
    import paper_1611_02274_amd as rk
    net = I.network_of("net13")
    y0, g = I.kinetics_inputs(net, 40, 9)
    yh, sh, sth = _host_run(rk.Problem.network(net), "rkc", y0, g, 0.0, 1e-6, 1e-8, 1e-12, 17)
    yo, so, sto = orc.rkc_batch(orc.network(net), y0, g, 0.0, 1e-6, 1e-8, 1e-12, max_steps=17)
    assert np.all(so == orc.MAXSTEPS)
    assert np.array_equal(sh, so) and np.array_equal(sth, sto) and np.array_equal(yh, yo)


@pytest.mark.parametrize("method,problem,n,seed,dt,k,rtol,atol,T_range", [
    ("rkc", "net13", 40, 2002, 1e-7, 6, 1e-8, 1e-12, (1000.0, 2500.0)),
    ("rkck", "net13", 24, 12, 5e-9, 5, 1e-8, 1e-12, (1000.0, 2500.0)),
    ("rkc", "vdp", 12, 3, 0.2, 8, 1e-8, 1e-10, None),
    ("rkck", "vdp", 12, 4, 0.2, 8, 1e-8, 1e-10, None),
    ("rkc", "net53", 6, 3003, 1e-7, 3, 1e-8, 1e-12, (900.0, 2800.0)),
])
def test_host_build_with_carried_state_equals_oracle(orc, method, problem, n, seed, dt, k, rtol,
                                                     atol, T_range):
    """Substeps with the controller state carried (the state modified between
    calls, as an operator-split transport step would): the kernels' host
    build reproduces the oracle's carried integration bit for bit, carried
    arrays included."""
    from paper_1611_02274_amd import _lib
    import paper_1611_02274_amd as rk
    if problem == "vdp":
        y0, g = I.vdp_inputs(n, seed)
        prob, pb = rk.Problem.vdp(), orc.vdp()
    else:
        net = I.network_of(problem)
        y0, g = I.kinetics_inputs(net, n, seed, T_range)
        prob, pb = rk.Problem.network(net), orc.network(net)
    f = _lib.lib().rkmi_test_host_integrate_carry
    f.argtypes = [C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                  C.c_double, C.c_double, C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                  C.c_int64, C.c_void_p]
    f.restype = C.c_int
    ch = orc.carry_init(pb, n)
    co = orc.carry_init(pb, n)
    yh = yo = np.ascontiguousarray(y0)
    g = np.ascontiguousarray(g)
    fo = orc.rkck_batch_carry if method == "rkck" else orc.rkc_batch_carry
    for s in range(k):
        y1 = np.zeros_like(yh)
        st = np.zeros(n, dtype=np.int32)
        stats = np.zeros((6, n), dtype=np.int32)
        assert f(0 if method == "rkck" else 1, prob.handle, n, yh.ctypes.data, y1.ctypes.data,
                 g.ctypes.data, s * dt, (s + 1) * dt, rtol, atol, st.ctypes.data,
                 stats.ctypes.data, 0, ch.ctypes.data) == 0
        yo1, so, sto = fo(pb, yo, g, co, s * dt, (s + 1) * dt, rtol, atol)
        assert np.array_equal(st, so) and np.array_equal(stats, sto)
        assert np.array_equal(y1.view(np.int64), yo1.view(np.int64))
        assert np.array_equal(ch.view(np.int64), co.view(np.int64))
        # a transport-like change of the state between substeps
        yh = yo = np.ascontiguousarray(yo1 * (1.0 + 1e-3 * np.cos(np.arange(n) + s)))
