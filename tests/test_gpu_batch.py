"""Ragged batches over the 9/13/32/53-species networks through the C ABI:
the persistent (queue-refilled) launch, the two plain forms and the captured
graph of substeps give the same bits, equal to the oracle run substep by
substep (each substep a restart over [k dt, (k + 1) dt])."""
import numpy as np
import pytest

from paper_1611_02274_amd import inputs as I

from .parity import compare, say

pytestmark = pytest.mark.gpu

SIZES = (9, 13, 32, 53)


@pytest.fixture(scope="module")
def rk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_02274_amd as rk
    return rk


def _setup(rk, n_total, seed, T_range=(800.0, 3000.0)):
    import torch
    slot_net, per_net = I.ragged_inputs(n_total, seed, T_range)
    nets = [I.standard_network(k) for k in SIZES]
    probs = [rk.Problem.network(n) for n in nets]
    batch = rk.Batch(probs)
    codes = torch.from_numpy(I.slot_map_codes(slot_net)).cuda()
    return nets, probs, batch, per_net, codes


def _buffers(per_net):
    import torch
    ys = [torch.from_numpy(y).cuda() for y, _ in per_net]
    gs = [torch.from_numpy(g).cuda() for _, g in per_net]
    st = [torch.empty(y.shape[1], dtype=torch.int32, device="cuda") for y in ys]
    stats = [torch.empty((6, y.shape[1]), dtype=torch.int32, device="cuda") for y in ys]
    return ys, gs, st, stats


def _run(rk, batch, per_net, codes, dt, n_sub, mode, bufs=None, **kw):
    import torch
    ys, gs, st, stats = bufs if bufs is not None else _buffers(per_net)
    if bufs is not None:
        for y, (y0, _) in zip(ys, per_net):
            y.copy_(torch.from_numpy(y0))
    batch.integrate_rkc(ys, gs, 0.0, dt, n_sub, 1e-8, 1e-12, mode=mode, slot_map=codes,
                        status=st, stats=stats, **kw)
    torch.cuda.synchronize()
    return ([y.cpu().numpy() for y in ys], [s.cpu().numpy() for s in st],
            [s.cpu().numpy() for s in stats])


def _oracle(orc, nets, per_net, dt, n_sub):
    out = []
    for net, (y0, g) in zip(nets, per_net):
        pb = orc.network(net)
        y = y0.copy()
        for k in range(n_sub):
            y, s, st = orc.rkc_batch(pb, y, g, 0.0 + k * dt, 0.0 + (k + 1) * dt, 1e-8, 1e-12)
        out.append((y, s, st))
    return out


def _same_bits(a, b):
    return all(np.array_equal(np.asarray(x).view(np.uint8), np.asarray(y).view(np.uint8))
               for x, y in zip(a, b))


def test_batch_modes_agree_and_equal_oracle(rk, orc):
    n_total, dt, n_sub = 3000, 2e-7, 3
    say(f"case batch modes n={n_total} dt={dt} substeps={n_sub}")
    nets, probs, batch, per_net, codes = _setup(rk, n_total, 11)
    res = {m: _run(rk, batch, per_net, codes, dt, n_sub, m)
           for m in ("persistent", "interleaved", "per_network")}
    for m in ("interleaved", "per_network"):
        for part in range(3):
            assert _same_bits(res[m][part], res["persistent"][part]), (m, part)
    ref = _oracle(orc, nets, per_net, dt, n_sub)
    for k, (yo, so, sto) in enumerate(ref):
        y, s, st = (res["persistent"][p][k] for p in range(3))
        compare(y, s, st, yo, so, sto, 1e-12, f"batch net{SIZES[k]}")


def test_batch_graph_replays(rk):
    """The captured graph of substeps, replayed (with eager work between the
    replays), gives the bits of the stream-ordered launches every time; a
    changed argument is captured anew."""
    import torch
    n_total, dt, n_sub = 2000, 2e-7, 4
    say(f"case batch graph n={n_total} substeps={n_sub}")
    nets, probs, batch, per_net, codes = _setup(rk, n_total, 5)
    eager = _run(rk, batch, per_net, codes, dt, n_sub, "persistent")
    bufs = _buffers(per_net)
    for rep in range(3):
        # the same buffers every time: the first call captures, the others replay
        got = _run(rk, batch, per_net, codes, dt, n_sub, "persistent", bufs=bufs, use_graph=True)
        for part in range(3):
            assert _same_bits(got[part], eager[part]), (rep, part)
        torch.ones(1000, device="cuda").sum().item()       # eager work between replays
    eager2 = _run(rk, batch, per_net, codes, dt, n_sub - 1, "persistent")
    got2 = _run(rk, batch, per_net, codes, dt, n_sub - 1, "persistent", bufs=bufs, use_graph=True)
    for part in range(3):
        assert _same_bits(got2[part], eager2[part])


def test_batch_schedule_options(rk):
    """Order, refill thresholds and grid size change the schedule, not the bits."""
    n_total, dt, n_sub = 2000, 2e-7, 2
    say("case batch schedule options")
    nets, probs, batch, per_net, codes = _setup(rk, n_total, 9)
    base = _run(rk, batch, per_net, codes, dt, n_sub, "persistent")
    for kw in (dict(order=[0, 1, 2, 3]), dict(refill=[1, 64, 8, 32]), dict(waves_per_cu=1)):
        got = _run(rk, batch, per_net, codes, dt, n_sub, "persistent", **kw)
        for part in range(3):
            assert _same_bits(got[part], base[part]), kw


def test_batch_carried_state(rk, orc):
    """Substeps with the controller state carried (per network [7 + N, n]
    arrays): the persistent launch, both plain forms and a replayed graph agree
    bit for bit, carried arrays included, and equal the oracle's carried
    substeps."""
    import torch
    n_total, dt, n_sub = 2000, 2e-7, 4
    say(f"case batch carry n={n_total} dt={dt} substeps={n_sub}")
    nets, probs, batch, per_net, codes = _setup(rk, n_total, 23)
    ref = []
    for net, (y0, g) in zip(nets, per_net):
        pb = orc.network(net)
        c = orc.carry_init(pb, y0.shape[1])
        y = y0.copy()
        for k in range(n_sub):
            y, s, st = orc.rkc_batch_carry(pb, y, g, c, k * dt, (k + 1) * dt, 1e-8, 1e-12)
        ref.append((y, s, st, c))
    outs = {}
    for mode, graph in (("persistent", False), ("interleaved", False), ("per_network", False),
                        ("persistent", True)):
        carry = [torch.zeros((rk.carry_rows(p), y.shape[1]), dtype=torch.float64, device="cuda")
                 for p, (y, _) in zip(probs, per_net)]
        ys, st, stats = _run(rk, batch, per_net, codes, dt, n_sub, mode, use_graph=graph,
                             carry=carry)
        outs[(mode, graph)] = (ys, st, stats, [c.cpu().numpy() for c in carry])
    base = outs[("persistent", False)]
    for key, o in outs.items():
        for a, b in zip(o, base):
            assert _same_bits(a, b), key
    for k, (yo, so, sto, co) in enumerate(ref):
        compare(base[0][k], base[1][k], base[2][k], yo, so, sto, 1e-12, f"carry net{SIZES[k]}")
        assert np.array_equal(base[3][k].view(np.int64), co.view(np.int64))
