"""Benchmark: batched FP64 ODE integration on one MI355X.

One step = one full integration of every system of the workload from t0 to t1
(all of the hot path: SoA load, rate setup, RHS, stages, error control,
power method, store), inputs resident in device memory.  Prints ONE JSON line.

    python bench.py [--steps K] [--warmup W] [--workload net53]

The default workload is the largest configuration: 2^20 systems of the
53-species network, one step = an RKCK integration and an RKC integration of
every system from the same initial states.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ODE systems integrated/sec at rtol 1e-8 (RKCK, RKC) vs FP64 roofline; adjoint grads/s"
FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 128 FP64 flop/clk x 2.4 GHz
# workloads whose step runs several methods over the same batch
COMBINED = {"net53": ("net53_rkck", "net53_rkc")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summaries
    (FETCH_SIZE, WRITE_SIZE scaled by a 1 GiB copy), or None when none matches
    this workload and the current kernel sources."""
    import glob

    from paper_1611_02274_amd.build import kernel_source_digest
    digest = kernel_source_digest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        kv = {}
        with open(path) as fh:
            for line in fh:
                parts = line.strip().split(":", 1)
                if len(parts) == 2 and parts[0].startswith(("traffic_", "kernel_source")):
                    kv[parts[0].strip()] = parts[1].strip()
        if kv.get("traffic_workload") == workload and kv.get("kernel_source_sha1") == digest:
            return float(kv["traffic_bytes_per_launch"]), os.path.basename(path)
    return None, None


def measured_ceilings():
    """Measured FP64 vector-ALU throughput (independent FMA chains; separate
    multiplies and adds, the mix of kernels that keep a*b + c unfused) and HBM
    bandwidth (a 1 GiB device-to-device copy, bytes read + written), reported
    beside the published peaks."""
    import ctypes

    import torch

    from paper_1611_02274_amd import _lib
    L = _lib.lib()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    out = torch.empty(int(L.rkmi_peak_threads()), dtype=torch.float64, device=dev)
    res = {}
    for mode, key in ((0, "fp64_fma_tflops"), (1, "fp64_mul_add_tflops")):
        fl = ctypes.c_double(0.0)
        best = 0.0
        for rep in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            _lib.check(L.rkmi_peak_fp64(mode, 20000, out.data_ptr(), ctypes.byref(fl),
                                        ctypes.c_void_p(stream.cuda_stream)))
            b.record(stream)
            torch.cuda.synchronize()
            if rep:
                best = max(best, fl.value / (a.elapsed_time(b) * 1e-3) / 1e12)
        res[key] = best
    x = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    best = 0.0
    for rep in range(4):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        y.copy_(x)
        b.record(stream)
        torch.cuda.synchronize()
        if rep:
            best = max(best, 2 * x.numel() * 8 / (a.elapsed_time(b) * 1e-3) / 1e9)
    res["hbm_copy_gbs"] = best
    res["published"] = {"fp64_vector_tflops": FP64_VECTOR_PEAK_TFLOPS, "hbm_gbs": 8000.0}
    del x, y, out
    return res


def cpu_baseline(parts, net, y0, g, target_s: float, sr_method: int = 0,
                 one_core_s: float = 5.0):
    """The oracle (serial per system, OpenMP across systems) on a bounded sample
    of the workload: every part (method) of a step integrates the same sampled
    systems; value = sampled systems / the parts' summed time.  Also the same on
    one core (the paper's serial baseline)."""
    import numpy as np

    from oracle import oracle as orc
    w0 = parts[0]
    pleiades = isinstance(net, str)
    thermal = w0.problem.endswith("_thermal")
    pb = (orc.vdp() if net is None else orc.pleiades() if pleiades
          else orc.network_thermal(net) if thermal else orc.network(net, sr_method))
    if net is None:
        pb = orc.vdp(sr_method)
    cores = orc.max_threads()

    def run(m, threads=0):
        idx = np.unique(np.linspace(0, w0.n - 1, m).astype(np.int64))
        t_all = 0.0
        for w in parts:
            fn = orc.rkck_batch if w.method == "rkck" else orc.rkc_batch
            ys = np.ascontiguousarray(y0[:, idx])
            gs = np.ascontiguousarray(g[:, idx]) if g is not None else None
            dt = (w.t1 - w.t0) / w.global_steps
            t = time.perf_counter()
            for k in range(w.global_steps):
                ys, _, _ = fn(pb, ys, gs, w.t0 + k * dt, w.t0 + (k + 1) * dt, w.rtol, w.atol,
                              n_threads=threads)
            t_all += time.perf_counter() - t
        return len(idx), t_all

    # a calibration sample large enough to average over the systems' costs and
    # the threads, then the sample sized to about target_s (once more if it fell
    # short of two thirds of that)
    m, dt = run(min(w0.n, max(64, 16 * cores)))
    for _ in range(2):
        if dt >= 0.66 * target_s or m >= w0.n:
            break
        want = int(m * target_s / max(dt, 1e-6))
        m, dt = run(min(w0.n, max(m + 1, want)))
    # one core: a sample sized to about one_core_s from the rate above
    m1 = max(4, min(w0.n, int(m / dt / cores * one_core_s)))
    m1, dt1 = run(m1, threads=1)
    what = " + ".join(w.method.upper() for w in parts)
    return {"value": m / dt, "unit": "systems/s", "cores": cores, "kind": "oracle",
            "sample": f"{m} of {w0.n} systems (evenly spaced), {what}, {dt:.1f} s on "
                      f"{cores} threads",
            "one_core": {"value": m1 / dt1, "unit": "systems/s", "cores": 1,
                         "sample": f"{m1} systems (evenly spaced), {what}, {dt1:.1f} s on "
                                   f"one thread"}}


def adjoint_bench(args, w, net):
    """One step = the taped forward (RKC, or RKCK for the _rkck workload) and
    the reverse sweep of the discrete adjoint (checkpoint every 16 accepted
    steps) for L = sum w . y(t1): the gradient of every system's loss with
    respect to y0 and ln A."""
    import numpy as np
    import torch

    import paper_1611_02274_amd as rk
    from paper_1611_02274_amd import flops as FL
    from paper_1611_02274_amd import inputs as I

    log(f"bench: adjoint workload {w.name} n={w.n}; generating inputs")
    y0, g = I.workload_inputs(w)
    wt = I.adjoint_weights(net.n_sp, w.n, w.seed)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prob = rk.Problem.network(net)
    yd, gd, wd = (torch.from_numpy(a).to(dev) for a in (y0, g, wt))
    ck = w.method == "rkck"
    K, cap = 16, (1024 if ck else 4096)
    taped = rk.integrate_rkck_taped if ck else rk.integrate_rkc_taped
    y1, st, stats, tape = taped(prob, yd, gd, w.t0, w.t1, w.rtol, w.atol, max_accepted=cap,
                                ckpt_every=K)
    torch.cuda.synchronize()
    if int(tape.count.min()) < 0:
        raise RuntimeError("tape too short for this workload")
    ms = int(stats[5].max())
    stream = torch.cuda.current_stream(dev)

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        taped(prob, yd, gd, w.t0, w.t1, w.rtol, w.atol, max_accepted=cap, ckpt_every=K, out=y1,
              status=st, stats=stats)
        if ev:
            ev[1].record(stream)
        out = (rk.adjoint_rkck(prob, gd, tape, wd) if ck
               else rk.adjoint_rkc(prob, gd, tape, wd, max_stages=ms))
        if ev:
            ev[2].record(stream)
        return out

    for k in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"bench: warmup {k + 1}/{args.warmup} done")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        dy0, dth, ast = step(evs[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fwd_ms = sum(e[0].elapsed_time(e[1]) for e in evs) / args.steps
    rev_ms = sum(e[1].elapsed_time(e[2]) for e in evs) / args.steps
    log(f"bench: {args.steps} steps in {elapsed:.3f} s; forward {fwd_ms:.3f} ms, "
        f"reverse {rev_ms:.3f} ms")
    st_h = stats.cpu().numpy()
    # accepted steps and their stage counts, from the tape
    n, cnt = w.n, tape.count.to(torch.int64)
    s_tab = tape.s
    mask = torch.arange(cap, device=dev)[:, None] < cnt[None, :]
    n_steps = float(cnt.sum())
    stage_sum = float((s_tab.to(torch.int64) * mask).sum())
    fwd_flops = FL.total(w.method, st_h, prob.n_eq, net)
    rev_flops = (FL.adjoint_reverse_rkck(prob.n_eq, net, n_steps) if ck
                 else FL.adjoint_reverse(prob.n_eq, net, n_steps, stage_sum))
    dom_ms, dom_flops, dom = ((rev_ms, rev_flops, "adjoint_kernel") if rev_ms >= fwd_ms
                              else (fwd_ms, fwd_flops, "taped_kernel"))
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12
    value = w.n * args.steps / elapsed
    res = {
        "metric": METRIC, "value": value, "unit": "grads/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "method": f"{w.method} discrete adjoint",
                   "problem": w.problem,
                   "n_systems": w.n, "t0": w.t0, "t1": w.t1, "rtol": w.rtol, "atol": w.atol,
                   "ckpt_every": K, "gradients": "dL/dy0 [13] and dL/dlnA [27] per system",
                   "schedule": "forward: plain, one system per lane (at 2^16 systems one "
                               "wave per SIMD: the cost order gains nothing); reverse: systems "
                               "in decreasing order of their taped step counts",
                   "systems_ok": int((ast.cpu().numpy() == 0).sum()),
                   "mean_accepted_steps": n_steps / w.n, "max_stages": ms},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": None, "kernel": dom, "kernel_ms": dom_ms,
                     "algorithmic_flops_per_launch": dom_flops,
                     "forward_ms": fwd_ms, "reverse_ms": rev_ms,
                     "forward_flops": fwd_flops, "reverse_flops": rev_flops},
    }
    if not args.no_cpu_baseline:
        log("bench: timing the oracle adjoint on a sample")
        from oracle import oracle as orc
        pb = orc.network(net)
        cores = orc.max_threads()

        def run(m):
            idx = np.unique(np.linspace(0, w.n - 1, m).astype(np.int64))
            a = [np.ascontiguousarray(x[:, idx]) for x in (y0, g, wt)]
            t = time.perf_counter()
            (orc.rkck_adjoint_batch if ck else orc.rkc_adjoint_batch)(
                pb, a[0], a[1], a[2], w.t0, w.t1, w.rtol, w.atol)
            return len(idx), time.perf_counter() - t

        m, dt = run(min(w.n, max(64, 8 * cores)))
        if dt < args.cpu_seconds and m < w.n:
            m, dt = run(min(w.n, max(m, int(m * args.cpu_seconds / max(dt, 1e-6)))))
        res["cpu_baseline"] = {"value": m / dt, "unit": "grads/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{m} of {w.n} systems (evenly spaced), {dt:.1f} s on "
                                         f"{cores} threads, store-everything adjoint",
                               "gpu_speedup": value / (m / dt)}
    print(json.dumps(res), flush=True)


def ragged_bench(args):
    """One step = n_substeps operator-splitting substeps of dt = 1e-6 s (each a
    restart, Sec. 3) over the ragged 10^6-system batch of the 9/13/32/53-species
    networks: the persistent launch per substep with the autotuned schedule,
    captured in one HIP graph.  Compared with one launch per network and
    substep on each network's own best schedule (group for 32/53 species,
    plain with the cost order for 9/13) over the same substeps, and, over the
    first --gate-substeps substeps, with the two plain forms (interleaved slots
    with a per-lane network switch; one plain launch per network)."""
    import numpy as np
    import torch

    import paper_1611_02274_amd as rk
    from paper_1611_02274_amd import autotune
    from paper_1611_02274_amd import flops as FL
    from paper_1611_02274_amd import inputs as I

    n_total = args.n or 1_000_000
    K, dt, rtol, atol = args.substeps, 1e-6, 1e-8, 1e-12
    G = min(K, args.gate_substeps)
    log(f"bench: ragged batch n={n_total}, {K} substeps; generating inputs")
    slot_net, per_net = I.ragged_inputs(n_total, 4004, (800.0, 3000.0))
    sizes = (9, 13, 32, 53)
    nets = [I.standard_network(k) for k in sizes]
    probs = [rk.Problem.network(n) for n in nets]
    batch = rk.Batch(probs)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    codes = torch.from_numpy(I.slot_map_codes(slot_net)).to(dev)
    y0 = [torch.from_numpy(y).to(dev) for y, _ in per_net]
    gs = [torch.from_numpy(g).to(dev) for _, g in per_net]
    ys = [y.clone() for y in y0]
    st = [torch.empty(y.shape[1], dtype=torch.int32, device=dev) for y in ys]
    stats = [torch.empty((6, y.shape[1]), dtype=torch.int32, device=dev) for y in ys]
    log("bench: autotuning the persistent schedule")
    tuned = autotune.tune_batch(batch, [y for y, _ in per_net], [g for _, g in per_net], dt, 1,
                                rtol, atol)
    log(f"bench: tuned {tuned}")

    # --carry: the controller state carried from substep to substep instead of
    # the restart (zeroed before every run, so each run starts with restarts)
    carry = ([torch.zeros((rk.carry_rows(p), y.shape[1]), dtype=torch.float64, device=dev)
              for p, y in zip(probs, ys)] if args.carry else None)

    def reset():
        for y, y_0 in zip(ys, y0):
            y.copy_(y_0)
        if carry is not None:
            for c in carry:
                c.zero_()
        torch.cuda.synchronize()

    def run(mode, n_sub, with_carry=True, **kw):
        reset()
        t = time.perf_counter()
        batch.integrate_rkc(ys, gs, 0.0, dt, n_sub, rtol, atol, mode=mode, slot_map=codes,
                            status=st, stats=stats, carry=carry if with_carry else None, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    # each network's own best single-network launch (no carried state)
    best = {9: dict(schedule=1, cost_order=1), 13: dict(schedule=1, cost_order=1),
            32: dict(schedule=3), 53: dict(schedule=3)}

    per_network_s = {}

    def run_separate(n_sub):
        reset()
        outs = [torch.empty_like(y) for y in ys]
        ev = []
        t = time.perf_counter()
        for j in range(n_sub):
            for k, (p, y, g) in enumerate(zip(probs, ys, gs)):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                rk.integrate_rkc(p, y, g, j * dt, (j + 1) * dt, rtol, atol, out=y, status=st[k],
                                 stats=stats[k], **best[sizes[k]])
                e1.record()
                ev.append((sizes[k], e0, e1))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t
        for size, e0, e1 in ev:
            per_network_s[str(size)] = per_network_s.get(str(size), 0.0) + e0.elapsed_time(e1) / 1e3
        del outs
        return elapsed

    times = {}
    for k in range(args.warmup):
        run("persistent", K, use_graph=True, **tuned)
        log(f"bench: warmup {k + 1}/{args.warmup} done")
    steps = []
    for k in range(args.steps):
        steps.append(run("persistent", K, use_graph=True, **tuned))
        log(f"bench: persistent graph {K} substeps {steps[-1]:.3f} s")
    times["persistent"] = min(steps)
    final = [y.cpu().numpy() for y in ys]
    ok = int(sum(int((s == 0).sum()) for s in st))
    status_counts = np.bincount(np.concatenate([s.cpu().numpy() for s in st]),
                                minlength=4).tolist()
    gate = {}
    if not args.carry and "separate" not in args.skip_modes.split(","):
        times["separate_best"] = run_separate(K)
        same = all(np.array_equal(a, b.cpu().numpy()) for a, b in zip(final, ys))
        log(f"bench: separate launches on each network's best schedule {times['separate_best']:.3f}"
            f" s, same bits as persistent: {same}; per network (s): "
            + ", ".join(f"{k} species {v:.3f}" for k, v in per_network_s.items()))
    if G > 0:
        gate["substeps"] = G
        gate["persistent_s"] = run("persistent", G, use_graph=True, **tuned)
        for mode in ("interleaved", "per_network"):
            if mode in args.skip_modes.split(","):
                continue
            gate[f"{mode}_s"] = run(mode, G)
            log(f"bench: first {G} substeps: {mode} {gate[f'{mode}_s']:.3f} s, persistent "
                f"{gate['persistent_s']:.3f} s")
        plain = [gate[f"{m}_s"] for m in ("interleaved", "per_network") if f"{m}_s" in gate]
        gate["speedup_vs_faster_plain"] = (min(plain) / gate["persistent_s"]) if plain else None
    if carry is not None:
        times["restart"] = run("persistent", K, with_carry=False, use_graph=True, **tuned)
        log(f"bench: persistent with restarts {times['restart']:.3f} s")
    # algorithmic flops: every substep's statistics (substeps one at a time, untimed)
    reset()
    flops = 0.0
    for k in range(K):
        batch.integrate_rkc(ys, gs, k * dt, dt, 1, rtol, atol, mode="persistent", status=st,
                            stats=stats, carry=carry, **tuned)
        torch.cuda.synchronize()
        flops += sum(FL.total("rkc", s.cpu().numpy(), n.n_sp, n) for s, n in zip(stats, nets))
    tp = times["persistent"]
    achieved = flops / tp / 1e12
    res = {
        "metric": METRIC, "value": n_total * K / tp, "unit": "system-substeps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": tp * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ragged_4net", "n_systems": n_total,
                   "networks": "9/19, 13/27, 32/133, 53/325 species/reactions, interleaved",
                   "substeps": K, "dt": dt, "rtol": rtol, "atol": atol, "method": "rkc",
                   "controller_state": "carried across substeps" if carry is not None
                                       else "restart at every substep",
                   "schedule": dict(mode="persistent (one launch per substep, HIP graph)",
                                    **tuned),
                   "systems_ok": ok, "status_counts": status_counts},
        "comparison": {"persistent_s": tp,
                       **{f"{m}_s": times[m] for m in times if m != "persistent"},
                       "speedup_vs_separate_best": (times["separate_best"] / tp
                                                    if "separate_best" in times else None),
                       "separate_best_schedules": {str(k): v for k, v in best.items()},
                       "separate_best_per_network_s": per_network_s or None},
        "gate": gate,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                     "traffic": None, "kernel": "ragged_kernel (whole graph)",
                     "algorithmic_flops_per_launch": flops / K},
    }
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 2 for the 2^20-system 53-species workloads, "
                         "else 10)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps (default: 1 for the 53-species workloads, else 2)")
    ap.add_argument("--workload", default="net53",
                    help="net53 (default: the 2^20-system 53-species batch under RKCK, then "
                         "RKC), or one of paper_1611_02274_amd.inputs.WORKLOADS, or ragged")
    ap.add_argument("--n", type=int, default=0,
                    help="systems (default: the workload's own count); for profiling runs")
    ap.add_argument("--substeps", type=int, default=100,
                    help="ragged workload: operator-splitting substeps per step")
    ap.add_argument("--gate-substeps", type=int, default=2,
                    help="ragged workload: substeps over which both plain forms are timed "
                         "against the persistent launch (0: none)")
    ap.add_argument("--carry", action="store_true",
                    help="ragged workload: carry the controller state across substeps")
    ap.add_argument("--skip-modes", default="",
                    help="ragged workload: comparisons not to run "
                         "(interleaved,per_network,separate)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the measured FP64 / HBM ceilings")
    ap.add_argument("--schedule", default="default",
                    choices=["default", "auto", "plain", "persistent", "group"],
                    help="default: the workload's own launch (schedule and cost order)")
    ap.add_argument("--cost-order", type=int, default=-1,
                    help="1: hand systems out in decreasing pilot cost; 0: queue order; "
                         "-1: the workload's own choice")
    ap.add_argument("--refill", type=int, default=0,
                    help="persistent schedule: idle lanes that trigger a refill (0: default)")
    ap.add_argument("--group-align", type=int, default=0,
                    help="group schedule: evaluations a group at its error estimate waits for "
                         "another group of its wave (0: the library default, < 0: never)")
    ap.add_argument("--sr-method", default="power", choices=("power", "gershgorin"),
                    help="RKC spectral radius: the nonlinear power method or the Gershgorin "
                         "bound of the analytic Jacobian (van der Pol, networks up to 16 species)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a device-to-device copy of 1 GiB, three times (the known "
                         "traffic that scales the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    big = args.workload.startswith(("net53", "net32")) or args.workload == "ragged"
    if args.steps is None:
        args.steps = (1 if args.workload == "ragged" else 2) if big else 10
    if args.warmup is None:
        args.warmup = 1 if big else 2
    if args.copy_calibration:
        import torch
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": x.numel() * 8, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the systems are "
              "independent, so a multi-GPU run is one shard per GPU with no exchange",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1611_02274_amd as rk
    from paper_1611_02274_amd import flops as FL
    from paper_1611_02274_amd import inputs as I

    if args.workload == "ragged":
        ragged_bench(args)
        return
    parts = [I.WORKLOADS[k] for k in COMBINED.get(args.workload, (args.workload,))]
    if args.n > 0:
        import dataclasses
        parts = [dataclasses.replace(p, n=args.n) for p in parts]
    w = parts[0]
    thermal = w.problem.endswith("_thermal")
    net = (None if w.problem == "vdp" else FL.PLEIADES if w.problem == "pleiades"
           else I.thermal_network(int(w.problem[3:-8])) if thermal else I.network_of(w.problem))
    if "_adjoint" in w.name:
        adjoint_bench(args, w, net)
        return
    log(f"bench: workload {args.workload} n={w.n}; generating inputs")
    y0, g = I.workload_inputs(w)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prob = (rk.Problem.vdp() if net is None else rk.Problem.pleiades() if net == FL.PLEIADES
            else rk.Problem.network_thermal(net) if thermal else rk.Problem.network(net))
    yd = torch.from_numpy(y0).to(dev)
    gd = torch.from_numpy(g).to(dev) if g is not None else None
    sched_names = {0: "automatic (group for more than 16 species, else persistent)",
                   1: "plain (one system per lane)",
                   2: "persistent (lanes refilled from a device queue)",
                   3: "group (several lanes per system, groups refilled from a device queue)"}

    class Part:
        """One method's integration of every system of the batch, [t0, t1] in
        w.global_steps global steps, each a restart (Sec. 3)."""

        def __init__(self, w):
            self.w = w
            self.out = torch.empty_like(yd)
            self.status = torch.empty(w.n, dtype=torch.int32, device=dev)
            self.stats = [torch.empty((rk.RK_NSTATS, w.n), dtype=torch.int32, device=dev)
                          for _ in range(w.global_steps)]
            self.fn = rk.integrate_rkck if w.method == "rkck" else rk.integrate_rkc
            launch = dict(w.launch)
            if args.schedule != "default":
                launch["schedule"] = {"auto": 0, "plain": 1, "persistent": 2,
                                      "group": 3}[args.schedule]
            if args.cost_order >= 0:
                launch["cost_order"] = args.cost_order
            if args.sr_method != "power":
                launch["sr_method"] = args.sr_method
            if args.refill:
                launch["refill"] = args.refill
            if args.group_align:
                launch["group_align"] = args.group_align
            self.launch = launch
            name = sched_names[launch.get("schedule", 0)]
            if launch.get("cost_order"):
                name += ("; cost order (a pilot at tolerances loosened 1e5 x, rtol at most "
                         "1e-3, counts each system's steps, systems handed out in decreasing "
                         "count; pilot and sort inside the timed step)")
            self.sched_name = name
            self.ms = []

        def run(self):
            w = self.w
            if w.global_steps == 1:
                self.fn(prob, yd, gd, w.t0, w.t1, w.rtol, w.atol, out=self.out,
                        status=self.status, stats=self.stats[0], **self.launch)
                return
            dt = (w.t1 - w.t0) / w.global_steps
            self.out.copy_(yd)
            for k in range(w.global_steps):
                self.fn(prob, self.out, gd, w.t0 + k * dt, w.t0 + (k + 1) * dt, w.rtol, w.atol,
                        out=self.out, status=self.status, stats=self.stats[k], **self.launch)

    P = [Part(p) for p in parts]
    stream = torch.cuda.current_stream(dev)

    def step(timed):
        for p in P:
            if timed:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                p.run()
                b.record(stream)
                p.ms.append((a, b))
            else:
                p.run()

    for k in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"bench: warmup {k + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for p in P:
        p.kern_ms = sum(a.elapsed_time(b) for a, b in p.ms) / args.steps
    log(f"bench: {args.steps} steps in {elapsed:.3f} s, kernels " +
        ", ".join(f"{p.w.name} {p.kern_ms:.3f} ms" for p in P))

    per = {}
    for p in P:
        st_all = [x.cpu().numpy() for x in p.stats]
        st_h = sum(x.astype(np.int64) for x in st_all)
        p.flops = sum(FL.total(p.w.method, x, prob.n_eq, FL.Thermal(net) if thermal else net)
                      for x in st_all)
        p.achieved = p.flops / (p.kern_ms * 1e-3) / 1e12
        per[p.w.name] = {
            "method": p.w.method, "schedule": p.sched_name, "launch": p.launch,
            "kernel_ms": p.kern_ms, "algorithmic_flops_per_launch": p.flops,
            "achieved_tflops": p.achieved, "frac": p.achieved / FP64_VECTOR_PEAK_TFLOPS,
            "systems_ok": int((p.status.cpu().numpy() == 0).sum()),
            "mean_accepted_steps": float(st_h[0].mean()),
            "mean_rejected_steps": float(st_h[1].mean()),
            "mean_rhs_evals": float(st_h[2].mean()),
            "max_stages": int(st_h[5].max()),
        }
    dom = max(P, key=lambda p: p.kern_ms)
    traffic, traffic_src = measured_traffic(dom.w.name + ("_gershgorin"
                                                          if dom.launch.get("sr_method") else ""))
    value = w.n * args.steps / elapsed
    n_global = dom.w.global_steps
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "systems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": args.workload, "methods": [p.w.method for p in P],
            "problem": w.problem, "n_systems": w.n, "t0": w.t0, "t1": w.t1, "rtol": w.rtol,
            "atol": w.atol, "global_steps": w.global_steps,
            "step": (" then ".join(f"{p.w.method.upper()} integration" for p in P) +
                     " of every system from the same initial states"),
            "parts": per,
        },
        "roofline": {
            "bound": "alu", "achieved": dom.achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": dom.achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": traffic, "traffic_unit": "bytes per launch",
            "traffic_source": traffic_src, "kernel": dom.w.name,
            "kernel_ms": dom.kern_ms, "algorithmic_flops_per_launch": dom.flops,
            "kernel_ms_covers": (("pilot, sort and integration kernels" if dom.launch.get(
                "cost_order") else "the integration kernel") +
                (f" of each of the {n_global} global-step calls" if n_global > 1
                 else " of one call")),
        },
    }
    if not args.no_ceilings:
        log("bench: measuring the FP64 and HBM ceilings")
        res["roofline"]["measured"] = measured_ceilings()
    if not args.no_cpu_baseline:
        log("bench: timing the oracle on a sample")
        res["cpu_baseline"] = cpu_baseline(parts, net, y0, g, args.cpu_seconds,
                                           1 if dom.launch.get("sr_method") == "gershgorin"
                                           else 0)
        res["cpu_baseline"]["gpu_speedup"] = value / res["cpu_baseline"]["value"]
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
