"""GPU discrete adjoint of RKC (taped forward + checkpointed reverse kernel)
through the C ABI, against the oracle's store-everything adjoint and against
central differences of the frozen step sequence."""
from concurrent.futures import ThreadPoolExecutor

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


def _gpu_adjoint(rk, prob, y0, g, w, t0, t1, rtol, atol, max_accepted=4096, ckpt_every=16):
    import torch
    yd = torch.from_numpy(y0).cuda()
    gd = torch.from_numpy(g).cuda()
    y1, st, stats, tape = rk.integrate_rkc_taped(prob, yd, gd, t0, t1, rtol, atol,
                                                 max_accepted=max_accepted,
                                                 ckpt_every=ckpt_every)
    dy0, dth, ast = rk.adjoint_rkc(prob, gd, tape, torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (y1, st, stats, dy0, dth, ast, tape.count)]


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("problem,n,t1,K", [("net13", 700, 1e-6, 16), ("net13", 130, 3e-7, 3),
                                            ("vdp", 300, 1.5, 16)])
def test_adjoint_equals_oracle(rk, orc, problem, n, t1, K):
    say(f"case adjoint {problem} n={n} t1={t1} K={K}")
    if problem == "vdp":
        y0, g = I.vdp_inputs(n, 17)
        prob, pb, atol = rk.Problem.vdp(), orc.vdp(), 1e-10
        w = np.random.default_rng(17).standard_normal((2, n))
    else:
        net = I.network_of(problem)
        y0, g = I.kinetics_inputs(net, n, 5005, (1000.0, 2500.0))
        prob, pb, atol = rk.Problem.network(net), orc.network(net), 1e-12
        w = I.adjoint_weights(net.n_sp, n, 5005)
    y1, st, stats, dy0, dth, ast, count = _gpu_adjoint(rk, prob, y0, g, w, 0.0, t1, 1e-8, atol,
                                                       max_accepted=20000, ckpt_every=K)
    yo, d0, dt, so = orc.rkc_adjoint_batch(pb, y0, g, w, 0.0, t1, 1e-8, atol)
    assert np.all(ast == 0) and np.array_equal(st, so)
    assert np.array_equal(count, stats[0])
    bitwise = float((dy0.view(np.int64) == d0.view(np.int64)).all(0).mean())
    say("adjoint parity", dict(dy0_rel=_rel(dy0, d0), dth_rel=_rel(dth, dt), bitwise=bitwise))
    assert _rel(y1, yo) <= 1e-9
    assert _rel(dy0, d0) <= 1e-9 and _rel(dth, dt) <= 1e-9


def _fd_system(orc, net, pb, gi, yi, wi, hs, ss, cols, e):
    """Central differences (absolute step e) of L = w . y(t1) over the frozen
    step sequence (hs, ss): d/dY0_m for every m, d/dlnA_j for j in cols."""
    def loss(p, y):
        return float(np.dot(wi, orc.rkc_replay(p, gi, y, 0.0, hs, ss)))
    fy = np.empty(len(yi))
    for m in range(len(yi)):
        d = np.zeros(len(yi))
        d[m] = e
        fy[m] = (loss(pb, yi + d) - loss(pb, yi - d)) / (2 * e)
    fa = np.empty(len(cols))
    for c, j in enumerate(cols):
        d = np.zeros(net.n_rx)
        d[j] = e
        fa[c] = (loss(pb.with_lnA(net.lnA + d), yi) - loss(pb.with_lnA(net.lnA - d), yi)) / (2 * e)
    return fy, fa


def test_adjoint_full_size_vs_oracle_and_fd(rk, orc):
    """The 2^16-system 13-species adjoint workload (checkpoint every 16 accepted
    steps) at full size; on 256 spread systems the gradients equal the
    oracle's adjoint, agree system by system to 1e-6 with complex-step
    derivatives of the frozen step sequence (every component of dL/dy0 and
    dL/dlnA; no cancellation, so each system is resolved on its own), and agree
    with central differences (h = 1e-6) of that sequence.  The differences carry
    a rounding error of a few 1e-9 (eps |L| / h, grown over ~10^3 steps), so
    their 1e-6 bar is taken over the 256 systems together (max norm per kind)."""
    w_ = I.WORKLOADS["net13_adjoint"]
    say(f"case adjoint full-size n={w_.n}")
    net = I.network_of(w_.problem)
    y0, g = I.workload_inputs(w_)
    w = I.adjoint_weights(net.n_sp, w_.n, w_.seed)
    prob, pb = rk.Problem.network(net), orc.network(net)
    y1, st, stats, dy0, dth, ast, count = _gpu_adjoint(rk, prob, y0, g, w, w_.t0, w_.t1, w_.rtol,
                                                       w_.atol)
    assert np.all(st == 0) and np.all(ast == 0) and np.all(count == stats[0])
    idx = np.unique(np.linspace(0, w_.n - 1, 256).astype(np.int64))
    ys, gs, ws = (np.ascontiguousarray(a[:, idx]) for a in (y0, g, w))
    yo, d0, dt, so = orc.rkc_adjoint_batch(pb, ys, gs, ws, w_.t0, w_.t1, w_.rtol, w_.atol)
    assert _rel(dy0[:, idx], d0) <= 1e-9 and _rel(dth[:, idx], dt) <= 1e-9
    cols = np.arange(0, net.n_rx, 3)
    n, nr = net.n_sp, net.n_rx

    def one(c):
        gi, yi, wi = gs[:, c], ys[:, c], ws[:, c]
        _, _, _, hs, ss = orc.rkc_solve(pb, gi, yi, w_.t0, w_.t1, w_.rtol, w_.atol)
        cy = np.array([orc.rkc_replay_jvp_cs(pb, gi, yi, w_.t0, hs, ss, wi, np.eye(n)[m])
                       for m in range(n)])
        ca = np.array([orc.rkc_replay_jvp_cs(pb, gi, yi, w_.t0, hs, ss, wi, np.zeros(n),
                                             np.eye(nr)[j]) for j in range(nr)])
        return cy, ca, _fd_system(orc, net, pb, gi, yi, wi, hs, ss, cols, 1e-6)

    with ThreadPoolExecutor(16) as ex:
        res = list(ex.map(one, range(len(idx))))
    ay, aa = dy0[:, idx], dth[:, idx]
    per_y = max(_rel(ay[:, c], r[0]) for c, r in enumerate(res))
    per_a = max(_rel(aa[:, c], r[1]) for c, r in enumerate(res))
    fy6 = np.stack([r[2][0] for r in res], 1)
    fa6 = np.stack([r[2][1] for r in res], 1)
    rel_y, rel_a = _rel(ay, fy6), _rel(aa[cols], fa6)
    say("adjoint vs complex step and FD",
        dict(systems=len(idx), dy0_rel_worst_system_cs=per_y, dlnA_rel_worst_system_cs=per_a,
             dy0_rel_fd_h1e6=rel_y, dlnA_rel_fd_h1e6=rel_a))
    assert per_y <= 1e-6 and per_a <= 1e-6
    assert rel_y <= 1e-6 and rel_a <= 1e-6


def test_autograd_function(rk):
    """rkc_solve: loss.backward() gives the adjoint kernel's gradients, the
    shared ln A gradient summed over systems; a tape too short is recorded
    again, longer."""
    import torch
    say("case autograd")
    net = I.network_of("net13")
    n = 200
    y0, g = I.kinetics_inputs(net, n, 31, (1000.0, 2500.0))
    w = torch.from_numpy(I.adjoint_weights(13, n, 31)).cuda()
    prob = rk.Problem.network(net)
    yd = torch.from_numpy(y0).cuda().requires_grad_(True)
    gd = torch.from_numpy(g).cuda()
    lnA = torch.from_numpy(net.lnA.copy()).cuda().requires_grad_(True)
    y1, st, stats = rk.rkc_solve(prob, yd, gd, 0.0, 1e-6, 1e-8, 1e-12, lnA=lnA, max_accepted=64)
    (w * y1).sum().backward()
    _, _, _, tape = rk.integrate_rkc_taped(prob, yd.detach(), gd, 0.0, 1e-6, 1e-8, 1e-12)
    dy0, dth, ast = rk.adjoint_rkc(prob, gd, tape, w)
    torch.cuda.synchronize()
    assert int(ast.abs().sum()) == 0
    assert torch.equal(yd.grad, dy0)
    assert torch.allclose(lnA.grad, dth.sum(1), rtol=1e-12, atol=0)
    # van der Pol: the gradient of mu arrives through g
    y0v, gv = I.vdp_inputs(64, 2)
    yv = torch.from_numpy(y0v).cuda().requires_grad_(True)
    gvd = torch.from_numpy(gv).cuda().requires_grad_(True)
    y1v, _, _ = rk.rkc_solve(rk.Problem.vdp(), yv, gvd, 0.0, 1.0, 1e-8, 1e-10)
    y1v.sum().backward()
    assert gvd.grad is not None and torch.isfinite(gvd.grad).all()
    assert torch.isfinite(yv.grad).all()


def test_tape_overflow_status(rk):
    import torch
    say("case tape overflow")
    net = I.network_of("net13")
    y0, g = I.kinetics_inputs(net, 100, 3, (1000.0, 2500.0))
    w = I.adjoint_weights(13, 100, 3)
    y1, st, stats, dy0, dth, ast, count = _gpu_adjoint(rk, rk.Problem.network(net), y0, g, w,
                                                       0.0, 1e-6, 1e-8, 1e-12, max_accepted=1000,
                                                       ckpt_every=16)
    over = stats[0] > 1000
    assert over.any() and (~over).any()
    assert np.all(count[over] == -1) and np.all(ast[over] == 4)
    assert np.all(np.isnan(dy0[:, over])) and np.all(np.isfinite(dy0[:, ~over]))
    assert np.all(ast[~over] == 0)


def _gpu_adjoint_rkck(rk, prob, y0, g, w, t0, t1, rtol, atol, max_accepted=4096, ckpt_every=16):
    import torch
    yd = torch.from_numpy(y0).cuda()
    gd = torch.from_numpy(g).cuda()
    y1, st, stats, tape = rk.integrate_rkck_taped(prob, yd, gd, t0, t1, rtol, atol,
                                                  max_accepted=max_accepted,
                                                  ckpt_every=ckpt_every)
    dy0, dth, ast = rk.adjoint_rkck(prob, gd, tape, torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (y1, st, stats, dy0, dth, ast, tape.count)]


@pytest.mark.parametrize("problem,n,t1,K", [("net13", 700, 5e-8, 16), ("net13", 130, 2e-8, 3),
                                            ("net9", 400, 5e-8, 8), ("vdp", 300, 2.0, 16)])
def test_rkck_adjoint_equals_oracle(rk, orc, problem, n, t1, K):
    """The RKCK discrete adjoint (taped forward, reverse sweep recomputing
    segments and stage arguments) against the oracle's store-everything RKCK
    adjoint, over several tiles and a ragged tail."""
    say(f"case rkck adjoint {problem} n={n} t1={t1} K={K}")
    if problem == "vdp":
        y0, g = I.vdp_inputs(n, 19)
        prob, pb, atol = rk.Problem.vdp(), orc.vdp(), 1e-10
        w = np.random.default_rng(19).standard_normal((2, n))
    else:
        net = I.network_of(problem)
        y0, g = I.kinetics_inputs(net, n, 5009, (1000.0, 2500.0))
        prob, pb, atol = rk.Problem.network(net), orc.network(net), 1e-12
        w = I.adjoint_weights(net.n_sp, n, 5009)
    y1, st, stats, dy0, dth, ast, count = _gpu_adjoint_rkck(rk, prob, y0, g, w, 0.0, t1, 1e-8,
                                                            atol, max_accepted=20000,
                                                            ckpt_every=K)
    yo, d0, dt, so = orc.rkck_adjoint_batch(pb, y0, g, w, 0.0, t1, 1e-8, atol)
    assert np.all(ast == 0) and np.array_equal(st, so)
    assert np.array_equal(count, stats[0])
    bitwise = float((dy0.view(np.int64) == d0.view(np.int64)).all(0).mean())
    say("rkck adjoint parity", dict(dy0_rel=_rel(dy0, d0), dth_rel=_rel(dth, dt), bitwise=bitwise))
    assert _rel(y1, yo) <= 1e-9
    assert _rel(dy0, d0) <= 1e-9 and _rel(dth, dt) <= 1e-9


def test_rkck_autograd_and_fd(rk, orc):
    """rkck_solve: loss.backward() gives the RKCK adjoint kernel's gradients;
    on a few systems they agree with central differences (h = 1e-6) of the
    frozen RKCK step sequence, normwise to 1e-6, and on every system, component
    by component, with complex-step derivatives of that sequence to 1e-6."""
    import torch
    say("case rkck autograd")
    net = I.network_of("net13")
    n = 96
    y0, g = I.kinetics_inputs(net, n, 37, (1000.0, 2500.0))
    w = I.adjoint_weights(13, n, 37)
    prob, pb = rk.Problem.network(net), orc.network(net)
    yd = torch.from_numpy(y0).cuda().requires_grad_(True)
    gd = torch.from_numpy(g).cuda()
    lnA = torch.from_numpy(net.lnA.copy()).cuda().requires_grad_(True)
    y1, st, stats = rk.rkck_solve(prob, yd, gd, 0.0, 5e-8, 1e-8, 1e-12, lnA=lnA, max_accepted=8)
    (torch.from_numpy(w).cuda() * y1).sum().backward()
    _, _, _, tape = rk.integrate_rkck_taped(prob, yd.detach(), gd, 0.0, 5e-8, 1e-8, 1e-12)
    dy0, dth, ast = rk.adjoint_rkck(prob, gd, tape, torch.from_numpy(w).cuda())
    torch.cuda.synchronize()
    assert int(ast.abs().sum()) == 0
    assert torch.equal(yd.grad, dy0)
    assert torch.allclose(lnA.grad, dth.sum(1), rtol=1e-12, atol=0)
    gy, ga = yd.grad.cpu().numpy(), dth.cpu().numpy()
    cols = np.arange(0, net.n_rx, 4)
    for i in (0, 41, 95):
        gi, yi, wi = g[:, i], y0[:, i], w[:, i]
        _, _, _, hs = orc.rkck_solve_rec(pb, gi, yi, 0.0, 5e-8, 1e-8, 1e-12)

        def loss(p, yy):
            return float(np.dot(wi, orc.rkck_replay(p, gi, yy, 0.0, hs)))
        e = 1e-6
        fy = np.array([(loss(pb, yi + e * np.eye(13)[m]) - loss(pb, yi - e * np.eye(13)[m])) / (2 * e)
                       for m in range(13)])
        fa = np.array([(loss(pb.with_lnA(net.lnA + e * np.eye(net.n_rx)[j]), yi) -
                        loss(pb.with_lnA(net.lnA - e * np.eye(net.n_rx)[j]), yi)) / (2 * e)
                       for j in cols])
        assert _rel(gy[:, i], fy) <= 1e-6
        assert _rel(ga[cols, i], fa) <= 1e-6

    def cs(i):
        gi, yi, wi = g[:, i], y0[:, i], w[:, i]
        _, _, _, hs = orc.rkck_solve_rec(pb, gi, yi, 0.0, 5e-8, 1e-8, 1e-12)
        cy = np.array([orc.rkck_replay_jvp_cs(pb, gi, yi, 0.0, hs, wi, np.eye(13)[m])
                       for m in range(13)])
        ca = np.array([orc.rkck_replay_jvp_cs(pb, gi, yi, 0.0, hs, wi, np.zeros(13),
                                              np.eye(net.n_rx)[j]) for j in range(net.n_rx)])
        return _rel(gy[:, i], cy), _rel(ga[:, i], ca)

    with ThreadPoolExecutor(16) as ex:
        worst = np.max(list(ex.map(cs, range(n))), axis=0)
    say("rkck adjoint vs complex step", dict(systems=n, dy0_rel_worst_system=worst[0],
                                             dlnA_rel_worst_system=worst[1]))
    assert worst[0] <= 1e-6 and worst[1] <= 1e-6


@pytest.mark.parametrize("method", ["rkc", "rkck"])
def test_taped_cost_order_changes_nothing(rk, method):
    """The taped forward with the cost order (pilot and sort in the tape's own
    working area) records the same tape and gives the same gradients bit for
    bit as the forward in system order."""
    import torch
    say(f"case taped cost order {method}")
    net = I.network_of("net13")
    n, t1 = 3000, (3e-7 if method == "rkc" else 5e-8)
    y0, g = I.kinetics_inputs(net, n, 5007, (1000.0, 2500.0))
    w = torch.from_numpy(I.adjoint_weights(net.n_sp, n, 5007)).cuda()
    prob = rk.Problem.network(net)
    yd, gd = torch.from_numpy(y0).cuda(), torch.from_numpy(g).cuda()
    taped = rk.integrate_rkc_taped if method == "rkc" else rk.integrate_rkck_taped
    adj = rk.adjoint_rkc if method == "rkc" else rk.adjoint_rkck
    outs = []
    for co in (0, 1):
        y1, st, stats, tape = taped(prob, yd, gd, 0.0, t1, 1e-8, 1e-12, max_accepted=2048,
                                    ckpt_every=16, cost_order=co)
        dy0, dth, ast = adj(prob, gd, tape, w)
        torch.cuda.synchronize()
        outs.append([x.cpu().numpy() for x in (y1, st, stats, tape.count, dy0, dth, ast)])
    for a, b in zip(*outs):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    assert np.all(outs[0][6] == 0)
