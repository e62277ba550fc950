"""The adjoint's per-system code (taped forward + reverse sweep with segment
and stage recomputation), compiled for the host from the kernels' source,
reproduces the oracle's store-everything adjoint bit for bit (CPU only)."""
import ctypes as C

import numpy as np
import pytest

from paper_1611_02274_amd import inputs as I


def _host_adjoint(prob, y0, g, w, t0, t1, rtol, atol, cap, K, max_stages=None, method=1):
    from paper_1611_02274_amd import _lib
    L = _lib.lib()
    n = y0.shape[1]
    L.rk_tape_bytes.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int32]
    L.rk_tape_bytes.restype = C.c_size_t
    nb = L.rk_tape_bytes(prob.handle, n, cap, K)
    assert nb > 0
    tape = np.zeros(nb + 256, dtype=np.uint8)
    base = tape.ctypes.data + (-tape.ctypes.data) % 256
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    y1 = np.zeros_like(y0)
    st = np.zeros(n, dtype=np.int32)
    stats = np.zeros((6, n), dtype=np.int32)
    f = L.rkmi_test_host_taped
    f.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                  C.c_double, C.c_double, C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                  C.c_void_p, C.c_size_t, C.c_int64, C.c_int32]
    assert f(prob.handle, method, n, y0.ctypes.data, y1.ctypes.data, g.ctypes.data, t0, t1, rtol, atol,
             st.ctypes.data, stats.ctypes.data, base, nb, cap, K) == 0
    ms = int(stats[5].max()) if max_stages is None else max_stages
    dy0 = np.zeros_like(y0)
    dth = np.zeros((prob.n_theta, n))
    ast = np.zeros(n, dtype=np.int32)
    fa = L.rkmi_test_host_adjoint
    fa.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p, C.c_size_t,
                   C.c_int64, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                   C.c_void_p]
    assert fa(prob.handle, method, n, g.ctypes.data, base, nb, cap, K, ms, w.ctypes.data,
              dy0.ctypes.data, dth.ctypes.data, ast.ctypes.data) == 0
    count = np.frombuffer(tape[base - tape.ctypes.data:][:4 * n].tobytes(), dtype=np.int32)
    return y1, st, stats, dy0, dth, ast, count


def _bits_equal(a, b):
    return np.array_equal(np.asarray(a).view(np.int64), np.asarray(b).view(np.int64))


@pytest.mark.parametrize("K", [16, 1, 5])
def test_network_adjoint_host_equals_oracle(orc, K):
    import paper_1611_02274_amd as rk
    net = I.network_of("net13")
    y0, g = I.kinetics_inputs(net, 20, 5005, (1000.0, 2500.0))
    w = I.adjoint_weights(13, 20, 5005)
    prob, pb = rk.Problem.network(net), orc.network(net)
    t1 = 1e-6 if K == 16 else 2e-7
    y1, st, stats, dy0, dth, ast, count = _host_adjoint(prob, y0, g, w, 0.0, t1, 1e-8, 1e-12,
                                                        cap=4096, K=K)
    yo, d0, dt, so = orc.rkc_adjoint_batch(pb, y0, g, w, 0.0, t1, 1e-8, 1e-12)
    assert np.all(ast == 0) and np.array_equal(st, so)
    assert np.array_equal(count, stats[0])
    assert _bits_equal(y1, yo)
    assert _bits_equal(dy0, d0)
    assert _bits_equal(dth, dt)


def test_vdp_adjoint_host_equals_oracle(orc):
    import paper_1611_02274_amd as rk
    y0, g = I.vdp_inputs(12, 3)
    w = np.random.default_rng(4).standard_normal((2, 12))
    prob, pb = rk.Problem.vdp(), orc.vdp()
    y1, st, stats, dy0, dth, ast, count = _host_adjoint(prob, y0, g, w, 0.0, 1.5, 1e-8, 1e-10,
                                                        cap=20000, K=16)
    yo, d0, dt, so = orc.rkc_adjoint_batch(pb, y0, g, w, 0.0, 1.5, 1e-8, 1e-10)
    assert np.all(ast == 0)
    assert _bits_equal(y1, yo) and _bits_equal(dy0, d0) and _bits_equal(dth, dt)


def test_tape_overflow_and_stage_bound_give_status_and_nan(orc):
    import paper_1611_02274_amd as rk
    net = I.network_of("net13")
    y0, g = I.kinetics_inputs(net, 6, 7, (1000.0, 2500.0))
    w = I.adjoint_weights(13, 6, 7)
    prob = rk.Problem.network(net)
    # a tape of 10 steps cannot hold these integrations
    y1, st, stats, dy0, dth, ast, count = _host_adjoint(prob, y0, g, w, 0.0, 1e-6, 1e-8, 1e-12,
                                                        cap=10, K=4)
    assert np.all(stats[0] > 10) and np.all(count == -1) and np.all(ast == 4)
    assert np.all(np.isnan(dy0)) and np.all(np.isnan(dth))
    yo, _, _, _ = orc.rkc_adjoint_batch(orc.network(net), y0, g, w, 0.0, 1e-6, 1e-8, 1e-12)
    assert _bits_equal(y1, yo)     # the forward result itself is unaffected
    # a stage bound below the recorded stage counts (hot 9-species systems
    # take 4-stage steps)
    net9 = I.network_of("net9")
    y0, g = I.kinetics_inputs(net9, 16, 7, (2000.0, 3000.0))
    w = I.adjoint_weights(9, 16, 7)
    y1, st, stats, dy0, dth, ast, count = _host_adjoint(rk.Problem.network(net9), y0, g, w, 0.0,
                                                        1e-6, 1e-8, 1e-12, cap=8192, K=16,
                                                        max_stages=2)
    big = stats[5] > 2
    assert big.any() and (~big).any()
    assert np.all(ast[big] == 4) and np.all(ast[~big] == 0)
    assert np.all(np.isnan(dy0[:, big])) and np.all(np.isfinite(dy0[:, ~big]))


@pytest.mark.parametrize("K", [16, 1, 3])
def test_rkck_network_adjoint_host_equals_oracle(orc, K):
    """RKCK: the taped forward and the reverse sweep (segments recomputed from
    checkpoints, stage arguments recomputed per step) on the host reproduce the
    oracle's store-everything RKCK adjoint bit for bit."""
    import paper_1611_02274_amd as rk
    net = I.network_of("net13")
    y0, g = I.kinetics_inputs(net, 12, 5007, (1000.0, 2500.0))
    w = I.adjoint_weights(13, 12, 5007)
    prob, pb = rk.Problem.network(net), orc.network(net)
    y1, st, stats, dy0, dth, ast, count = _host_adjoint(prob, y0, g, w, 0.0, 3e-8, 1e-8, 1e-12,
                                                        cap=4096, K=K, method=0)
    yo, d0, dt, so = orc.rkck_adjoint_batch(pb, y0, g, w, 0.0, 3e-8, 1e-8, 1e-12)
    assert np.all(ast == 0) and np.array_equal(st, so)
    assert np.array_equal(count, stats[0]) and count.min() >= 1 and count.max() > 10
    assert _bits_equal(y1, yo)
    assert _bits_equal(dy0, d0)
    assert _bits_equal(dth, dt)


def test_rkck_vdp_adjoint_host_equals_oracle(orc):
    import paper_1611_02274_amd as rk
    y0, g = I.vdp_inputs(10, 5)
    w = np.random.default_rng(6).standard_normal((2, 10))
    prob, pb = rk.Problem.vdp(), orc.vdp()
    y1, st, stats, dy0, dth, ast, count = _host_adjoint(prob, y0, g, w, 0.0, 2.0, 1e-8, 1e-10,
                                                        cap=20000, K=7, method=0)
    yo, d0, dt, so = orc.rkck_adjoint_batch(pb, y0, g, w, 0.0, 2.0, 1e-8, 1e-10)
    assert np.all(ast == 0)
    assert _bits_equal(y1, yo) and _bits_equal(dy0, d0) and _bits_equal(dth, dt)
