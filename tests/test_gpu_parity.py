"""GPU parity: the HIP kernels through the C ABI against the CPU oracle,
element by element on the same seeded inputs."""
import numpy as np
import pytest

from paper_1611_02274_amd import inputs as I

from .parity import compare, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_02274_amd as rk
    return rk


def _gpu(rk, method, prob, y0, g, t0, t1, rtol, atol, **kw):
    import torch
    yd = torch.from_numpy(y0).cuda()
    gd = torch.from_numpy(g).cuda() if g is not None else None
    fn = rk.integrate_rkck if method == "rkck" else rk.integrate_rkc
    y1, st, stats = fn(prob, yd, gd, t0, t1, rtol, atol, **kw)
    torch.cuda.synchronize()
    return y1.cpu().numpy(), st.cpu().numpy(), stats.cpu().numpy()


def _orc(orc, method, pb, y0, g, t0, t1, rtol, atol, **kw):
    fn = orc.rkck_batch if method == "rkck" else orc.rkc_batch
    return fn(pb, y0, g, t0, t1, rtol, atol, **kw)


def _case(rk, orc, method, problem, n, seed, t0, t1, rtol, atol, T_range=(1000.0, 2500.0), **kw):
    say(f"case {method} {problem} n={n} seed={seed} t=[{t0},{t1}] rtol={rtol} atol={atol}")
    if problem in ("vdp", "vdp_stiff"):
        y0, g = I.vdp_inputs(n, seed, (300.0, 3000.0) if problem == "vdp_stiff" else (0.5, 2.0))
        prob, pb = rk.Problem.vdp(), orc.vdp()
    else:
        net = I.network_of(problem)
        y0, g = I.kinetics_inputs(net, n, seed, T_range)
        prob, pb = rk.Problem.network(net), orc.network(net)
    yg, sg, stg = _gpu(rk, method, prob, y0, g, t0, t1, rtol, atol, **kw)
    oo = {k: v for k, v in kw.items() if k == "max_steps"}
    yo, so, sto = _orc(orc, method, pb, y0, g, t0, t1, rtol, atol, **oo)
    return compare(yg, sg, stg, yo, so, sto, atol, f"{method}/{problem}/n={n}")


def test_vdp_rkck_full(rk, orc):
    """4096 van der Pol oscillators, RKCK, t in [0, 10], rtol 1e-8, atol 1e-10."""
    _case(rk, orc, "rkck", "vdp", 4096, 1, 0.0, 10.0, 1e-8, 1e-10)


def test_vdp_rkc_ragged(rk, orc):
    _case(rk, orc, "rkc", "vdp", 1000, 3, 0.0, 2.0, 1e-8, 1e-10)


@pytest.mark.parametrize("n", [1, 63, 65, 4133])
def test_net13_rkc(rk, orc, n):
    _case(rk, orc, "rkc", "net13", n, 2002, 0.0, 1e-6, 1e-8, 1e-12)


def test_net9_rkc(rk, orc):
    _case(rk, orc, "rkc", "net9", 2000, 77, 0.0, 1e-6, 1e-8, 1e-12, T_range=(800.0, 3000.0))


def test_net13_rkck(rk, orc):
    _case(rk, orc, "rkck", "net13", 700, 12, 0.0, 2e-8, 1e-8, 1e-12)


@pytest.mark.parametrize("schedule", [1, 2])
def test_vdp_rkc_stiff_many_stages(rk, orc, schedule):
    """Steps of 10 to 60 stages: lanes of a wave read tabulated coefficients
    (up to 32 stages) or form them, side by side."""
    _case(rk, orc, "rkc", "vdp_stiff", 1000, 13, 0.0, 1.0, 1e-6, 1e-8, schedule=schedule)


@pytest.mark.parametrize("problem,n,schedule,cost_order", [
    ("vdp_stiff", 1000, 1, 0), ("vdp", 777, 2, 0), ("net13", 4133, 1, 0), ("net13", 4133, 2, 0),
    ("net13", 2000, 1, 1), ("net9", 1000, 0, 0)])
def test_rkc_gershgorin(rk, orc, problem, n, schedule, cost_order):
    """RKC with the Gershgorin bound of the analytic Jacobian in place of the
    power method equals the oracle bit for bit under every schedule."""
    import torch
    say(f"case gershgorin {problem} n={n} schedule={schedule} cost_order={cost_order}")
    if problem.startswith("vdp"):
        y0, g = I.vdp_inputs(n, 13, (300.0, 3000.0) if problem == "vdp_stiff" else (0.5, 2.0))
        prob, pb = rk.Problem.vdp(), orc.vdp(orc.SR_GERSHGORIN)
        t1, rtol, atol = 1.0, 1e-6, 1e-8
    else:
        net = I.network_of(problem)
        y0, g = I.kinetics_inputs(net, n, 2002, (900.0, 2800.0))
        prob, pb = rk.Problem.network(net), orc.network(net, orc.SR_GERSHGORIN)
        t1, rtol, atol = 1e-6, 1e-8, 1e-12
    yd, gd = torch.from_numpy(y0).cuda(), torch.from_numpy(g).cuda()
    y1, st, stats = rk.integrate_rkc(prob, yd, gd, 0.0, t1, rtol, atol, sr_method="gershgorin",
                                     schedule=schedule, cost_order=cost_order)
    torch.cuda.synchronize()
    yo, so, sto = orc.rkc_batch(pb, y0, g, 0.0, t1, rtol, atol)
    compare(y1.cpu().numpy(), st.cpu().numpy(), stats.cpu().numpy(), yo, so, sto, atol,
            f"gershgorin {problem}")
    assert np.all(sto[4] == 0)


def test_gershgorin_rejected_without_a_jacobian(rk):
    """Problems without an analytic Jacobian and taped integrations refuse the
    option (RK_EUNSUPPORTED) rather than falling back."""
    import torch
    y0, _ = I.pleiades_inputs(4, 6006)
    yd = torch.from_numpy(y0).cuda()
    with pytest.raises(RuntimeError):
        rk.integrate_rkc(rk.Problem.pleiades(), yd, None, 0.0, 0.1, 1e-8, 1e-10,
                         sr_method="gershgorin")
    net = I.network_of("net53")
    y0, g = I.kinetics_inputs(net, 4, 1, (900.0, 2800.0))
    with pytest.raises(RuntimeError):
        rk.integrate_rkc(rk.Problem.network(net), torch.from_numpy(y0).cuda(),
                         torch.from_numpy(g).cuda(), 0.0, 1e-7, 1e-8, 1e-12,
                         sr_method="gershgorin")


def test_vdp_rkck_loose_and_tight(rk, orc):
    _case(rk, orc, "rkck", "vdp", 777, 5, 0.0, 3.0, 1e-5, 0.0)
    _case(rk, orc, "rkck", "vdp", 777, 6, 0.0, 3.0, 1e-11, 1e-13)


def test_max_steps_status(rk, orc):
    _case(rk, orc, "rkc", "net13", 300, 9, 0.0, 1e-6, 1e-8, 1e-12, max_steps=17)
    _case(rk, orc, "rkck", "vdp", 300, 9, 0.0, 10.0, 1e-8, 1e-10, max_steps=40)


def test_nonfinite_input_status(rk, orc):
    """A NaN initial state is rejected until the step underflows hMin, on both sides."""
    say("case nan vdp")
    y0, g = I.vdp_inputs(130, 4)
    y0[:, 7] = np.nan
    y0[1, 100] = np.inf
    prob, pb = rk.Problem.vdp(), orc.vdp()
    for m in ("rkck", "rkc"):
        yg, sg, stg = _gpu(rk, m, prob, y0, g, 0.0, 1.0, 1e-8, 1e-10)
        yo, so, sto = _orc(orc, m, pb, y0, g, 0.0, 1.0, 1e-8, 1e-10)
        assert sg[7] != 0 and np.array_equal(sg, so)
        ok = np.isfinite(yo).all(0)
        compare(yg[:, ok], sg[ok], stg[:, ok], yo[:, ok], so[ok], sto[:, ok], 1e-10, f"nan/{m}")


def test_empty_interval_and_in_place(rk):
    import torch
    say("case empty interval / in place")
    y0, g = I.vdp_inputs(100, 2)
    prob = rk.Problem.vdp()
    yd, gd = torch.from_numpy(y0).cuda(), torch.from_numpy(g).cuda()
    y1, st, stats = rk.integrate_rkck(prob, yd, gd, 1.0, 1.0, 1e-8, 1e-10)
    torch.cuda.synchronize()
    assert torch.equal(y1, yd) and int(st.abs().sum()) == 0 and int(stats.abs().sum()) == 0
    ref, _, _ = rk.integrate_rkck(prob, yd, gd, 0.0, 1.0, 1e-8, 1e-10)
    inplace = yd.clone()
    rk.integrate_rkck(prob, inplace, gd, 0.0, 1.0, 1e-8, 1e-10, out=inplace)
    torch.cuda.synchronize()
    assert torch.equal(inplace, ref)
    # zero systems is a no-op
    e = torch.empty((2, 0), dtype=torch.float64, device="cuda")
    rk.integrate_rkc(prob, e, torch.empty((1, 0), dtype=torch.float64, device="cuda"),
                     0.0, 1.0, 1e-8, 1e-10)


def test_argument_errors(rk):
    import ctypes as C
    import torch
    from paper_1611_02274_amd import _lib
    say("case argument errors")
    prob = rk.Problem.vdp()
    y = torch.zeros((2, 8), dtype=torch.float64, device="cuda")
    g = torch.ones((1, 8), dtype=torch.float64, device="cuda")
    L = _lib.lib()
    f = L.rk_integrate_rkc

    def call(n=8, y0=y.data_ptr(), y1=y.data_ptr(), gg=g.data_ptr(), t0=0.0, t1=1.0, rtol=1e-6,
             atol=0.0):
        return f(prob.handle, n, y0, y1, gg, t0, t1, rtol, atol, None, None, None, 0, None, None)

    assert call(n=-1) == _lib.RK_EINVAL
    assert call(t1=-1.0) == _lib.RK_EINVAL
    assert call(rtol=0.0) == _lib.RK_EINVAL
    assert call(atol=-1.0) == _lib.RK_EINVAL
    assert call(t1=float("nan")) == _lib.RK_EINVAL
    host = np.zeros(16)
    assert call(y0=host.ctypes.data) == _lib.RK_EINVAL
    assert b"not" in L.rk_last_error()
    assert call(y0=y.data_ptr() + 4) == _lib.RK_EINVAL
    assert call(gg=None) == _lib.RK_EINVAL
    assert f(None, 8, y.data_ptr(), y.data_ptr(), g.data_ptr(), 0.0, 1.0, 1e-6, 0.0, None, None,
             None, 0, None, None) == _lib.RK_EINVAL
    assert call() == _lib.RK_OK
    # options: a group alignment is accepted (it only concerns group launches);
    # a nonzero reserved word is refused
    o = rk._options(schedule=1, group_align=3)
    assert f(prob.handle, 8, y.data_ptr(), y.data_ptr(), g.data_ptr(), 0.0, 1.0, 1e-6, 0.0, None,
             None, None, 0, C.byref(o), None) == _lib.RK_OK
    o.reserved[2] = 1
    assert f(prob.handle, 8, y.data_ptr(), y.data_ptr(), g.data_ptr(), 0.0, 1.0, 1e-6, 0.0, None,
             None, None, 0, C.byref(o), None) == _lib.RK_EINVAL
    assert b"reserved" in L.rk_last_error()
    torch.cuda.synchronize()


@pytest.mark.parametrize("wname,n_sample", [("net13_rkc", 512), ("net53_rkc", 256),
                                           ("net53_rkck", 256)])
def test_full_size_sampled(rk, orc, wname, n_sample):
    """The 2^18-system 13-species RKC and the 2^20-system 53-species RKC / RKCK
    workloads at full size, in the launch the benchmark times; the oracle
    recomputes a spread sample of systems."""
    w = I.WORKLOADS[wname]
    say(f"case full-size {w.name} n={w.n}")
    net = I.network_of(w.problem)
    y0, g = I.workload_inputs(w)
    prob, pb = rk.Problem.network(net), orc.network(net)
    yg, sg, stg = _gpu(rk, w.method, prob, y0, g, w.t0, w.t1, w.rtol, w.atol, **w.launch)
    idx = np.unique(np.linspace(0, w.n - 1, n_sample).astype(np.int64))
    yo, so, sto = _orc(orc, w.method, pb, np.ascontiguousarray(y0[:, idx]),
                       np.ascontiguousarray(g[:, idx]), w.t0, w.t1, w.rtol, w.atol)
    compare(yg[:, idx], sg[idx], stg[:, idx], yo, so, sto, w.atol, f"full {w.name} sample")
    # whole-batch properties: every system finished, mass fractions still sum to one
    assert np.all(sg == 0)
    assert np.abs(yg.sum(0) - 1.0).max() < 1e-11


def test_device_math_equals_host_and_oracle(rk, orc):
    """The correctly rounded exp / log / pow give the same bits on the device as
    the host build of the same source, and as the oracle."""
    import ctypes as C
    import torch
    from paper_1611_02274_amd import _lib
    say("case device math")
    L = _lib.lib()
    fd, fh = L.rkmi_crmath_device, L.rkmi_crmath_host
    fd.argtypes = [C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    fh.argtypes = [C.c_int, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
    rng = np.random.default_rng(11)
    n = 200_000
    cases = [(0, rng.uniform(-45, 45, n), np.zeros(n)),
             (1, rng.uniform(300, 4000, n), np.zeros(n)),
             (2, 10 ** rng.uniform(-20, 3, n), np.full(n, -0.2)),
             (2, 10 ** rng.uniform(-20, 3, n), np.full(n, 2.0 / 3.0)),
             (3, 10 ** rng.uniform(-30, 6, n), np.zeros(n)),
             (4, 10 ** rng.uniform(-30, 6, n), np.zeros(n)),
             (5, 10 ** rng.uniform(-30, 6, n), np.zeros(n)),
             (6, 10 ** rng.uniform(-30, 6, n), np.zeros(n)),
             (7, 10 ** rng.uniform(-30, 6, n), np.zeros(n))]
    ref = {0: orc.cr_exp, 1: orc.cr_log, 3: lambda v, w: orc.cr_pow(v, 1.0 / 3.0),
           4: lambda v, w: orc.cr_pow(v, 2.0 / 3.0), 5: lambda v, w: orc.cr_pow(v, 1.0 / 3.0),
           6: lambda v, w: orc.cr_pow(v, -0.25), 7: lambda v, w: orc.cr_pow(v, -0.2)}
    for fn, x, y in cases:
        xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
        od = torch.empty_like(xd)
        assert fd(fn, n, xd.data_ptr(), yd.data_ptr(), od.data_ptr(), None) == 0
        torch.cuda.synchronize()
        oh = np.zeros(n)
        assert fh(fn, n, x.ctypes.data, y.ctypes.data, oh.ctypes.data) == 0
        dev = od.cpu().numpy()
        assert np.array_equal(dev, oh), (fn, int((dev != oh).sum()))
        m = 20000
        r = np.array([ref[fn](v) if fn < 2 else ref.get(fn, orc.cr_pow)(v, w)
                      for v, w in zip(x[:m], y[:m])])
        assert np.array_equal(dev[:m], r)


@pytest.mark.parametrize("problem,method,n,t1,T_range", [
    ("net13", "rkc", 5000, 1e-6, (1000.0, 2500.0)),
    ("net9", "rkc", 3000, 1e-6, (800.0, 3000.0)),
    ("net13", "rkck", 800, 2e-8, (1000.0, 2500.0)),
    ("vdp", "rkck", 3000, 10.0, None),
    # vectors and rate constants in workspace columns
    ("net53", "rkc", 700, 1e-6, (900.0, 2800.0)),
    ("net53", "rkck", 700, 1e-6, (900.0, 2800.0)),
    ("net32", "rkc", 700, 1e-6, (900.0, 2800.0)),
    ("net32", "rkck", 300, 1e-6, (900.0, 2800.0)),
])
def test_schedules_agree_bitwise(rk, orc, problem, method, n, t1, T_range):
    """The plain, the persistent (queue-refilled) and the group (16 lanes per
    system, for the 32- and 53-species networks) schedules, each with and
    without the cost order, give identical bits (the group one also with every
    phase alignment), and all equal the oracle."""
    import torch
    say(f"case schedules {problem} {method} n={n}")
    if problem == "vdp":
        y0, g = I.vdp_inputs(n, 21)
        prob, pb, atol = rk.Problem.vdp(), orc.vdp(), 1e-10
    else:
        net = I.network_of(problem)
        y0, g = I.kinetics_inputs(net, n, 21, T_range)
        prob, pb, atol = rk.Problem.network(net), orc.network(net), 1e-12
    res = [_gpu(rk, method, prob, y0, g, 0.0, t1, 1e-8, atol, schedule=s, cost_order=co)
           for co in (0, 1) for s in (1, 2, 3)]
    if problem in ("net32", "net53"):
        # the group schedule with no phase alignment and a long one
        res += [_gpu(rk, method, prob, y0, g, 0.0, t1, 1e-8, atol, schedule=3, group_align=a)
                for a in (-1, 8)]
    for other in res[1:]:
        for a, b in zip(res[0], other):
            assert np.array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8))
    yo, so, sto = _orc(orc, method, pb, y0, g, 0.0, t1, 1e-8, atol)
    compare(*res[1], yo, so, sto, atol, f"persistent {method}/{problem}")


def test_column_workspace(rk, orc):
    """Systems held in workspace columns: too small a workspace is refused with
    RK_EWORKSPACE (plain and persistent); a workspace of one workgroup block
    runs a one-workgroup persistent grid with the same bits as the full one."""
    import ctypes as C
    import torch
    from paper_1611_02274_amd import _lib
    say("case column workspace")
    net = I.network_of("net53")
    y0, g = I.kinetics_inputs(net, 200, 8, (900.0, 2800.0))
    prob = rk.Problem.network(net)
    L = _lib.lib()
    yd, gd = torch.from_numpy(y0).cuda(), torch.from_numpy(g).cuda()
    ref, st_ref, stats_ref = rk.integrate_rkc(prob, yd, gd, 0.0, 1e-6, 1e-8, 1e-12)
    opt = _lib.Options()
    opt.schedule = 2
    full = L.rk_workspace_bytes(prob.handle, 1, 200, C.byref(opt))
    assert full > 256
    opt.schedule = 1
    plain = L.rk_workspace_bytes(prob.handle, 1, 200, C.byref(opt))
    block = (plain - 256) // 4          # 200 systems = 4 workgroups
    assert plain == 256 + 4 * block
    out = torch.empty_like(yd)
    st = torch.empty(200, dtype=torch.int32, device="cuda")
    stats = torch.empty((6, 200), dtype=torch.int32, device="cuda")
    ws = torch.empty(plain, dtype=torch.uint8, device="cuda")

    def call(schedule, nbytes):
        opt.schedule = schedule
        return L.rk_integrate_rkc(prob.handle, 200, yd.data_ptr(), out.data_ptr(), gd.data_ptr(),
                                  0.0, 1e-6, 1e-8, 1e-12, st.data_ptr(), stats.data_ptr(),
                                  ws.data_ptr(), nbytes, C.byref(opt), None)

    assert call(1, plain - 8) == _lib.RK_EWORKSPACE
    assert call(2, 256 + block - 8) == _lib.RK_EWORKSPACE
    assert call(2, 256 + block) == _lib.RK_OK
    torch.cuda.synchronize()
    assert torch.equal(out, ref) and torch.equal(st, st_ref) and torch.equal(stats, stats_ref)
    assert call(1, plain) == _lib.RK_OK
    torch.cuda.synchronize()
    assert torch.equal(out, ref) and torch.equal(stats, stats_ref)


@pytest.mark.parametrize("n", [1, 63, 65, 4097])
def test_cost_order_in_place(rk, orc, n):
    """The cost order integrating in place (the pilot must leave y0 alone) over
    ragged sizes, plain and persistent, equals the oracle."""
    import torch
    say(f"case cost order in place n={n}")
    net = I.network_of("net13")
    y0, g = I.kinetics_inputs(net, n, 31, (1000.0, 2500.0))
    prob = rk.Problem.network(net)
    yo, so, sto = _orc(orc, "rkc", orc.network(net), y0, g, 0.0, 2e-7, 1e-8, 1e-12)
    for s in (1, 2):
        yd, gd = torch.from_numpy(y0).cuda(), torch.from_numpy(g).cuda()
        y1, st, stats = rk.integrate_rkc(prob, yd, gd, 0.0, 2e-7, 1e-8, 1e-12, out=yd,
                                         schedule=s, cost_order=1)
        torch.cuda.synchronize()
        assert y1.data_ptr() == yd.data_ptr()
        compare(y1.cpu().numpy(), st.cpu().numpy(), stats.cpu().numpy(), yo, so, sto, 1e-12,
                f"cost order in place s={s} n={n}")


def test_cost_order_rejects(rk):
    """The cost order needs its workspace and is refused for a taped integration."""
    import ctypes as C

    import torch
    from paper_1611_02274_amd import _lib
    L = _lib.lib()
    net = I.network_of("net13")
    y0, g = I.kinetics_inputs(net, 100, 1, (1000.0, 2500.0))
    prob = rk.Problem.network(net)
    yd, gd = torch.from_numpy(y0).cuda(), torch.from_numpy(g).cuda()
    out = torch.empty_like(yd)
    o = rk._options(schedule=1, cost_order=1)
    need = L.rk_workspace_bytes(prob.handle, _lib.RK_METHOD_RKC, 100, C.byref(o))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    f = L.rk_integrate_rkc
    assert f(prob.handle, 100, yd.data_ptr(), out.data_ptr(), gd.data_ptr(), 0.0, 1e-7, 1e-8,
             1e-12, None, None, ws.data_ptr(), need - 256, C.byref(o), s) == _lib.RK_EWORKSPACE
    assert f(prob.handle, 100, yd.data_ptr(), out.data_ptr(), gd.data_ptr(), 0.0, 1e-7, 1e-8,
             1e-12, None, None, ws.data_ptr(), need, C.byref(o), s) == _lib.RK_OK
    torch.cuda.synchronize()


def _pleiades_global_steps(fn_step, y0, n_global=10, t0=0.0, t1=1.0):
    """Ten global steps over [t0, t1], each a restart (Sec. 4.1)."""
    y, dt, last = y0, (t1 - t0) / n_global, None
    for k in range(n_global):
        y, st, stats = fn_step(y, t0 + k * dt, t0 + (k + 1) * dt)
        last = (st, stats)
    return y, last[0], last[1]


@pytest.mark.parametrize("n,schedule,cost_order", [(4133, 1, 0), (4133, 2, 0), (1000, 1, 1),
                                                   (65, 2, 1), (4133, 3, 0), (1000, 3, 1),
                                                   (65, 0, 0), (9, 3, 0)])
def test_pleiades_rkck(rk, orc, n, schedule, cost_order):
    """The Pleiades problem under RKCK at eps = 1e-10 over the ten global
    steps of [0, 1]: one lane per system with 28 unknowns in workspace columns
    (plain, persistent) and eight lanes per system (group, the default), each
    equal to the oracle step by step."""
    import torch
    say(f"case pleiades n={n} schedule={schedule} cost_order={cost_order}")
    y0, _ = I.pleiades_inputs(n, 6006)
    prob, pb = rk.Problem.pleiades(), orc.pleiades()

    def gpu_step(y, a, b):
        yd = torch.from_numpy(np.ascontiguousarray(y)).cuda()
        y1, st, stats = rk.integrate_rkck(prob, yd, None, a, b, 1e-10, 0.0, out=yd,
                                          schedule=schedule, cost_order=cost_order)
        torch.cuda.synchronize()
        return y1.cpu().numpy(), st.cpu().numpy(), stats.cpu().numpy()

    def orc_step(y, a, b):
        return orc.rkck_batch(pb, y, None, a, b, 1e-10, 0.0)

    yg, sg, stg = _pleiades_global_steps(gpu_step, y0)
    yo, so, sto = _pleiades_global_steps(orc_step, y0)
    compare(yg, sg, stg, yo, so, sto, 1e-10, f"pleiades n={n}")


@pytest.mark.parametrize("schedule", [1, 3])
def test_pleiades_rkc(rk, orc, schedule):
    """RKC on the Pleiades problem (one global step of 0.1): the group
    variant's RKC driver and the one-lane kernel equal the oracle."""
    say(f"case pleiades rkc schedule={schedule}")
    import torch
    y0, _ = I.pleiades_inputs(700, 6008)
    prob, pb = rk.Problem.pleiades(), orc.pleiades()
    yd = torch.from_numpy(y0).cuda()
    y1, st, stats = rk.integrate_rkc(prob, yd, None, 0.0, 0.1, 1e-8, 1e-10, schedule=schedule)
    torch.cuda.synchronize()
    yo, so, sto = orc.rkc_batch(pb, y0, None, 0.0, 0.1, 1e-8, 1e-10)
    compare(y1.cpu().numpy(), st.cpu().numpy(), stats.cpu().numpy(), yo, so, sto, 1e-10,
            f"pleiades rkc schedule={schedule}")


def test_pleiades_full_size_sampled(rk, orc):
    """The 2^18-system Pleiades workload in the benchmark's launch: ten global
    steps on the GPU; the oracle recomputes a spread sample of 256 systems."""
    import torch
    w = I.WORKLOADS["pleiades_rkck"]
    say(f"case full-size {w.name} n={w.n}")
    y0, _ = I.workload_inputs(w)
    prob, pb = rk.Problem.pleiades(), orc.pleiades()
    yd = torch.from_numpy(y0).cuda()

    def gpu_step(y, a, b):
        y1, st, stats = rk.integrate_rkck(prob, y, None, a, b, w.rtol, w.atol, out=y, **w.launch)
        return y1, st, stats
    yg, sg, stg = _pleiades_global_steps(gpu_step, yd, t0=w.t0, t1=w.t1)
    torch.cuda.synchronize()
    yg, sg, stg = yg.cpu().numpy(), sg.cpu().numpy(), stg.cpu().numpy()
    idx = np.unique(np.linspace(0, w.n - 1, 256).astype(np.int64))
    yo, so, sto = _pleiades_global_steps(
        lambda y, a, b: orc.rkck_batch(pb, y, None, a, b, w.rtol, w.atol),
        np.ascontiguousarray(y0[:, idx]), t0=w.t0, t1=w.t1)
    compare(yg[:, idx], sg[idx], stg[:, idx], yo, so, sto, 1e-10, "full pleiades sample")
    assert np.all(sg == 0)


@pytest.mark.parametrize("problem,method,n,dt,k,schedules", [
    ("net13", "rkc", 3000, 2e-7, 4, (1, 2)),
    ("net13", "rkck", 1500, 1e-8, 4, (1, 2)),
    ("net53", "rkc", 400, 2e-7, 3, (1, 3)),
    ("net32", "rkck", 300, 5e-8, 3, (2, 3)),
    ("vdp", "rkck", 2000, 0.5, 6, (1, 2)),
])
def test_carried_state_equals_oracle(rk, orc, problem, method, n, dt, k, schedules):
    """Substeps with the controller state carried between calls and the state
    perturbed between them: every schedule (one lane or a group per system,
    with and without the cost order) gives the oracle's bits, carried arrays
    included."""
    import torch
    say(f"case carry {problem} {method} n={n} substeps={k}")
    if problem == "vdp":
        y0, g = I.vdp_inputs(n, 41)
        prob, pb, atol = rk.Problem.vdp(), orc.vdp(), 1e-10
    else:
        net = I.network_of(problem)
        y0, g = I.kinetics_inputs(net, n, 41, (900.0, 2800.0))
        prob, pb, atol = rk.Problem.network(net), orc.network(net), 1e-12
    fo = orc.rkck_batch_carry if method == "rkck" else orc.rkc_batch_carry
    fg = rk.integrate_rkck if method == "rkck" else rk.integrate_rkc

    def bump(y, s):
        return np.ascontiguousarray(y * (1.0 + 1e-3 * np.cos(np.arange(y.shape[1]) + s)))

    co = orc.carry_init(pb, n)
    yo = y0
    for s in range(k):
        yo1, so, sto = fo(pb, yo, g, co, s * dt, (s + 1) * dt, 1e-8, atol)
        yo = bump(yo1, s)
    gd = torch.from_numpy(g).cuda()
    for sched in schedules:
        for cost in (0, 1):
            cg = torch.zeros((rk.carry_rows(prob), n), dtype=torch.float64, device="cuda")
            yg = y0
            for s in range(k):
                y1, st, stats = fg(prob, torch.from_numpy(yg).cuda(), gd, s * dt, (s + 1) * dt,
                                   1e-8, atol, schedule=sched, cost_order=cost, carry=cg)
                torch.cuda.synchronize()
                yg1 = y1.cpu().numpy()
                yg = bump(yg1, s)
            compare(yg1, st.cpu().numpy(), stats.cpu().numpy(), yo1, so, sto, atol,
                    f"carry {problem} {method} schedule={sched} cost={cost}")
            assert np.array_equal(cg.cpu().numpy().view(np.int64), co.view(np.int64))


@pytest.mark.parametrize("n_sp,method,n,t1,schedule,cost_order", [
    (13, "rkc", 4133, 1e-6, 1, 0), (13, "rkc", 4133, 1e-6, 2, 1), (9, "rkc", 2000, 1e-6, 2, 0),
    (13, "rkck", 700, 5e-8, 1, 1),
    # 32 and 53 species + T: the group kernels (32 lanes per system) under every
    # schedule, the last group of a wave partly filled (odd n)
    (32, "rkc", 67, 1e-8, 3, 0), (32, "rkck", 97, 1e-8, 1, 1), (53, "rkc", 37, 1e-8, 3, 1),
    (53, "rkc", 33, 5e-9, 2, 0), (53, "rkck", 67, 1e-8, 3, 0)])
def test_thermal_networks(rk, orc, n_sp, method, n, t1, schedule, cost_order):
    """Networks with the energy equation (state T, Y; rate coefficients at the
    current T): every schedule equals the oracle; up to 15 species on the
    one-lane kernels, above on the group kernels whatever the schedule."""
    say(f"case thermal net{n_sp} {method} n={n} schedule={schedule} cost={cost_order}")
    net = I.thermal_network(n_sp)
    y0, g = I.thermal_inputs(net, n, 8100 + n_sp, (1000.0, 2500.0))
    prob, pb = rk.Problem.network_thermal(net), orc.network_thermal(net)
    yg, sg, stg = _gpu(rk, method, prob, y0, g, 0.0, t1, 1e-8, 1e-12, schedule=schedule,
                       cost_order=cost_order)
    yo, so, sto = _orc(orc, method, pb, y0, g, 0.0, t1, 1e-8, 1e-12)
    compare(yg, sg, stg, yo, so, sto, 1e-12, f"thermal net{n_sp} {method}")


@pytest.mark.parametrize("wname,n_sample", [("net13_thermal_rkc", 128),
                                           ("net53_thermal_rkc", 16)])
def test_thermal_full_size_sampled(rk, orc, wname, n_sample):
    """The 2^18-system workloads with the energy equation in the benchmark's
    launch: 13 species over ten global steps of 1e-6 s (one-lane kernels), 53
    species over one (group kernels); the oracle recomputes a spread sample."""
    import torch
    w = I.WORKLOADS[wname]
    say(f"case full-size {w.name} n={w.n}")
    net = I.thermal_network(int(w.problem[3:-8]))
    y0, g = I.workload_inputs(w)
    prob, pb = rk.Problem.network_thermal(net), orc.network_thermal(net)
    yd, gd = torch.from_numpy(y0).cuda(), torch.from_numpy(g).cuda()
    dt = (w.t1 - w.t0) / w.global_steps
    for k in range(w.global_steps):
        y1, st, stats = rk.integrate_rkc(prob, yd, gd, w.t0 + k * dt, w.t0 + (k + 1) * dt, w.rtol,
                                         w.atol, out=yd, **w.launch)
    torch.cuda.synchronize()
    yg, sg, stg = yd.cpu().numpy(), st.cpu().numpy(), stats.cpu().numpy()
    idx = np.unique(np.linspace(0, w.n - 1, n_sample).astype(np.int64))
    yo = np.ascontiguousarray(y0[:, idx])
    gs = np.ascontiguousarray(g[:, idx])
    for k in range(w.global_steps):
        yo, so, sto = orc.rkc_batch(pb, yo, gs, w.t0 + k * dt, w.t0 + (k + 1) * dt, w.rtol, w.atol)
    compare(yg[:, idx], sg[idx], stg[:, idx], yo, so, sto, w.atol, f"full {w.name} sample")
    assert np.all(sg == 0)
    assert np.abs(yg[1:].sum(0) - 1.0).max() < 1e-11
