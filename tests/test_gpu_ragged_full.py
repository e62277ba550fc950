"""The ragged batch at its stated size: 1,000,000 interleaved systems of the
9/13/32/53-species networks (T ~ U[800, 3000] K, seed 4004), 100
operator-splitting substeps of 1e-6 s captured in one HIP graph of persistent
launches, each substep a restart (Sec. 3: a new integration per global step).
A seeded sample of systems from every network, plus every system the launch
stopped with a non-OK status, is recomputed by the oracle substep by substep;
final state, status and the last substep's statistics are compared."""
import numpy as np
import pytest

from paper_1611_02274_amd import inputs as I

from .parity import compare, say

pytestmark = pytest.mark.gpu

SIZES = (9, 13, 32, 53)
N_TOTAL, SEED, DT, N_SUB = 1_000_000, 4004, 1e-6, 100
RTOL, ATOL = 1e-8, 1e-12
PER_NET_SAMPLE = 24


@pytest.fixture(scope="module")
def rk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1611_02274_amd as rk
    return rk


def test_ragged_full_size_against_oracle(rk, orc):
    import torch
    say(f"case ragged full size n={N_TOTAL} substeps={N_SUB} dt={DT} (graph, persistent)")
    slot_net, per_net = I.ragged_inputs(N_TOTAL, SEED, (800.0, 3000.0))
    nets = [I.standard_network(k) for k in SIZES]
    probs = [rk.Problem.network(n) for n in nets]
    batch = rk.Batch(probs)
    ys = [torch.from_numpy(y).cuda() for y, _ in per_net]
    gs = [torch.from_numpy(g).cuda() for _, g in per_net]
    st = [torch.empty(y.shape[1], dtype=torch.int32, device="cuda") for y in ys]
    stats = [torch.empty((6, y.shape[1]), dtype=torch.int32, device="cuda") for y in ys]
    batch.integrate_rkc(ys, gs, 0.0, DT, N_SUB, RTOL, ATOL, mode="persistent", status=st,
                        stats=stats, use_graph=True)
    torch.cuda.synchronize()
    say("ragged full size: GPU done")
    rng = np.random.default_rng(4005)
    for k, (net, (y0, g)) in enumerate(zip(nets, per_net)):
        n = y0.shape[1]
        s_gpu = st[k].cpu().numpy()
        bad = np.flatnonzero(s_gpu != 0)
        idx = np.unique(np.concatenate([rng.choice(n, PER_NET_SAMPLE, replace=False), bad]))
        say(f"ragged full size net{SIZES[k]}: {idx.size} systems sampled, "
            f"{bad.size} non-OK on the GPU {np.bincount(s_gpu, minlength=4).tolist()}")
        pb = orc.network(net)
        y = np.ascontiguousarray(y0[:, idx])
        gg = np.ascontiguousarray(g[:, idx])
        for j in range(N_SUB):
            y, so, sto = orc.rkc_batch(pb, y, gg, j * DT, (j + 1) * DT, RTOL, ATOL)
        compare(ys[k].cpu().numpy()[:, idx], s_gpu[idx], stats[k].cpu().numpy()[:, idx], y, so,
                sto, ATOL, f"ragged full size net{SIZES[k]}")
