"""Schedule autotuner for batched integration.

Picks, by timing candidates on a seeded sample of the workload, the schedule
of one network (plain / persistent / group, refill threshold, cost order,
group alignment) or of a ragged
batch (network order, per-network refill thresholds, workgroups per compute
unit).  Results are cached per (network topologies, method, rtol, device) in a
JSON file, so a workload is tuned once per machine.  Every candidate computes
the same bits (the schedules only change which lane runs which system when),
so tuning never changes results.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

CACHE_ENV = "RKMI_TUNE_CACHE"


def _cache_path() -> str:
    p = os.environ.get(CACHE_ENV)
    if p:
        return p
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "paper_1611_02274_amd", "tune.json")


def _load() -> dict:
    try:
        with open(_cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(key: str, value: dict) -> None:
    path = _cache_path()
    data = _load()
    data[key] = value
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".{os.getpid()}"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass                      # a read-only cache only costs a re-tune


def _device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(p, 'gcnArchName', p.name)}/{p.multi_processor_count}cu"


def _time(fn, reps: int = 2) -> float:
    import torch
    fn()                          # warm (first launch, graph capture)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t)
    return best


def sample_indices(n: int, fraction: float, minimum: int, seed: int) -> np.ndarray:
    """Seeded sample of max(minimum, fraction * n) systems, in index order."""
    m = min(n, max(minimum, int(round(fraction * n))))
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=m, replace=False))


NETWORK_CANDIDATES = (
    dict(schedule=1),                                   # plain, one lane per system
    dict(schedule=2, refill=8), dict(schedule=2, refill=16), dict(schedule=2, refill=32),
    dict(schedule=3, refill=16), dict(schedule=3, refill=32),   # group (large networks)
    # group: how long a group at its error estimate waits for the other groups
    # of its wave (never; longer than the default)
    dict(schedule=3, refill=32, group_align=-1), dict(schedule=3, refill=32, group_align=8),
    # systems handed out in decreasing cost (a loose-tolerance pilot ranks them)
    dict(schedule=1, cost_order=1), dict(schedule=2, refill=16, cost_order=1),
)


def tune_network(problem, method: str, y0, g, t0, t1, rtol, atol, fraction=0.05,
                 minimum=16384, seed=0, force=False) -> dict:
    """Best schedule for integrating this network: returns the keyword
    arguments for integrate_rkck / integrate_rkc (schedule, refill, cost order,
    group alignment)."""
    import torch

    from . import integrate_rkc, integrate_rkck
    topo = problem.net.topology_key() if problem.net is not None else problem.kind
    key = f"net/{topo}/{method}/{rtol:g}/{_device_key()}"
    cached = _load().get(key)
    if cached and not force:
        return cached["best"]
    idx = sample_indices(y0.shape[1], fraction, minimum, seed)
    ys = torch.from_numpy(np.ascontiguousarray(y0[:, idx])).cuda()
    gs = torch.from_numpy(np.ascontiguousarray(g[:, idx])).cuda()
    fn = integrate_rkck if method == "rkck" else integrate_rkc
    out = torch.empty_like(ys)
    cands = [c for c in NETWORK_CANDIDATES
             if (c["schedule"] != 3 or problem.n_eq > 16) and (not c.get("cost_order") or
                                                               c["schedule"] != 3)]
    times = []
    for c in cands:
        times.append(_time(lambda: fn(problem, ys, gs, t0, t1, rtol, atol, out=out, **c)))
    best = cands[int(np.argmin(times))]
    _store(key, {"best": best, "sample": int(len(idx)),
                 "times": {json.dumps(c, sort_keys=True): t for c, t in zip(cands, times)}})
    return best


def tune_batch(batch, ys, gs, dt, n_sub, rtol, atol, fraction=0.05, minimum=16384, seed=0,
               force=False) -> dict:
    """Best persistent-batch schedule (order, refill per network, workgroups per
    compute unit) on a seeded sample of each network's systems; returns the
    keyword arguments for Batch.integrate_rkc."""
    import itertools

    import torch
    probs = batch.problems
    topo = "+".join(p.net.topology_key() for p in probs)
    key = f"batch/{topo}/rkc/{rtol:g}/{_device_key()}"
    cached = _load().get(key)
    if cached and not force:
        return cached["best"]
    samples = []
    for k, (y, g) in enumerate(zip(ys, gs)):
        idx = sample_indices(y.shape[1], fraction, minimum // len(probs), seed + k)
        samples.append((np.ascontiguousarray(y[:, idx]), np.ascontiguousarray(g[:, idx])))
    dev_y = [torch.from_numpy(y).cuda() for y, _ in samples]
    dev_g = [torch.from_numpy(g).cuda() for _, g in samples]
    work = [y.clone() for y in dev_y]
    heavy = list(np.argsort([-p.n_eq for p in probs]))
    orders = [heavy, heavy[::-1]]
    cands = []
    for order, refill, wpc in itertools.product(orders, (8, 16, 32), (0, 2)):
        cands.append(dict(order=[int(o) for o in order], refill=[refill] * len(probs),
                          waves_per_cu=wpc))

    def run(c):
        for w, y in zip(work, dev_y):
            w.copy_(y)
        batch.integrate_rkc(work, dev_g, 0.0, dt, n_sub, rtol, atol, mode="persistent", **c)

    times = [_time(lambda: run(c)) for c in cands]
    best = cands[int(np.argmin(times))]
    _store(key, {"best": best, "samples": [int(y.shape[1]) for y, _ in samples],
                 "times": {json.dumps(c, sort_keys=True): t for c, t in zip(cands, times)}})
    return best
