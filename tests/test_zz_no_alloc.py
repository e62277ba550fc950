"""The allocation-free RKC entry point (rk_integrate_rkc_noalloc, workspace in the
library's own device array) through the C ABI: the same bits as
rk_integrate_rkc with a caller-allocated workspace, on two calls in a row (the
second smaller, so it runs on what the first left in the shared array), for
schedules whose kernels use the workspace (queue head, cost order's pilot
statistics, order map and histogram); a call needing more than the array
returns RK_EWORKSPACE and enqueues nothing."""
import ctypes as C

import numpy as np
import pytest

from paper_1611_02274_amd import inputs as I

from .parity import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_02274_amd as rk
    return rk


def _call(rk, fn, prob, y0, g, t1, opt, ws=None):
    """One call of `fn` (rk_integrate_rkc or rk_integrate_rkc_noalloc) on
    device copies of y0, g; returns (rc, y1, status, stats) on the host."""
    import torch
    L = rk._lib.lib()
    n = y0.shape[1]
    yd = torch.from_numpy(y0).cuda()
    gd = torch.from_numpy(g).cuda()
    y1 = torch.full_like(yd, -7.0)
    st = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    stats = torch.full((6, n), -7, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    args = [prob.handle, n, yd.data_ptr(), y1.data_ptr(), gd.data_ptr(), 0.0, t1, 1e-8, 1e-12,
            st.data_ptr(), stats.data_ptr()]
    if fn == "rk_integrate_rkc":
        nws = L.rk_workspace_bytes(prob.handle, rk._lib.RK_METHOD_RKC, n, C.byref(opt))
        wsb = torch.empty(max(nws, 1), dtype=torch.uint8, device="cuda")
        rc = L.rk_integrate_rkc(*args, wsb.data_ptr() if nws else None, nws, C.byref(opt), s)
    else:
        rc = L.rk_integrate_rkc_noalloc(*args, C.byref(opt), s)
    torch.cuda.synchronize()
    return rc, y1.cpu().numpy(), st.cpu().numpy(), stats.cpu().numpy()


@pytest.mark.parametrize("problem,schedule,cost_order", [
    ("net13", 1, 1),    # plain + cost order: pilot statistics, order map, histogram
    ("net13", 2, 0),    # persistent: the queue head
    ("net53", 3, 1),    # group + cost order
])
def test_noalloc_equals_workspace_entry(rk, problem, schedule, cost_order):
    net = I.network_of(problem)
    prob = rk.Problem.network(net)
    opt = rk._lib.Options()
    opt.schedule, opt.cost_order = schedule, cost_order
    t1 = 1e-6 if problem == "net13" else 1e-7
    for n, seed in ((4133, 61), (1000, 62)):      # the second call smaller
        say(f"case noalloc {problem} schedule={schedule} cost_order={cost_order} n={n}")
        y0, g = I.kinetics_inputs(net, n, seed, (1000.0, 2500.0))
        ref = _call(rk, "rk_integrate_rkc", prob, y0, g, t1, opt)
        got = _call(rk, "rk_integrate_rkc_noalloc", prob, y0, g, t1, opt)
        assert ref[0] == 0 and got[0] == 0, rk._lib.lib().rk_last_error()
        assert np.all(ref[2] == 0)
        for a, b in zip(ref[1:], got[1:]):
            assert np.array_equal(a, b)


def test_noalloc_rejects_oversized_workspace(rk):
    """The 53-species one-lane plain kernel keeps its vectors in workspace
    columns (about 6 KB per system): 2^14 systems need more than the array."""
    net = I.network_of("net53")
    prob = rk.Problem.network(net)
    opt = rk._lib.Options()
    opt.schedule = 1
    L = rk._lib.lib()
    n = 1 << 14
    assert L.rk_workspace_bytes(prob.handle, rk._lib.RK_METHOD_RKC, n,
                                C.byref(opt)) > rk._lib.RK_SCRATCH_BYTES
    y0, g = I.kinetics_inputs(net, n, 63, (1000.0, 2500.0))
    rc, y1, st, stats = _call(rk, "rk_integrate_rkc_noalloc", prob, y0, g, 1e-7, opt)
    assert rc == rk._lib.RK_EWORKSPACE
    assert b"allocation-free" in L.rk_last_error()
    assert np.all(y1 == -7.0) and np.all(st == -7)      # nothing was enqueued
