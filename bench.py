"""Benchmark: exact LOO log-likelihood pair-kernel evaluations per second.

Default workload (N=1 GPU): gradient ascent on the photoz-shaped set,
N = 500,000, dx = 5, dy = 1, diagonal (per-dimension) bandwidths.  One step
is one evaluation of the exact LOO log-likelihood and its bandwidth gradient
(one O(N^2) pass of the adjoint kernel over all ordered pairs i != j) plus
the Adam update of theta = log h on the host.  Pair-kernel evaluations per
step: N (N - 1).

Prints one JSON line with the throughput, the roofline of the dominant
kernel (timed live with HIP events on the stream it runs on) and the FP64
CPU oracle timed on a bounded sample of the same workload.  Secondary
figures, measured after the timed steps: the value-only pass, one density
query batch on the same resident set (16,384 queries x 256 grid points,
fraction of the FP32 matrix-core peak) and a short serving stream in both
modes.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Peak FP32 vector rate of MI355X in lane-operations per second: 256 CUs x
# 4 SIMDs x 2.4 GHz x 32 lanes (the published 157.3 TFLOP/s counts an FMA as
# two FLOPs).  Non-packed FP32 instructions reach it by dual issue: each SIMD
# issues two wave64 VALU instructions (from different waves) per 4-cycle
# quad; a probe measured 2.4-2.6 cycles per wave64 FMA at 4-8 waves/SIMD.
VALU_PEAK_SLOTS = 256 * 4 * 32 * 2.4e9
# Issue cost of one v_exp_f32 in those FP32 slots: the transcendental rate is
# a quarter of the dual-issue FP32 rate (8 lanes/clock/SIMD; the probe
# measured 9.7 cycles per wave64 exp, 83% of that).
EXP_SLOTS = 4.0
# Algorithmic FP32 work per ordered pair of the value+gradient pass (dx=5,
# dy=1): 6 differences, 6 squares, 6 exponent FMAs, 2 kernel-sum adds and 11
# moment FMAs (F = 31), plus two exponentials (E = 2).  The kernel issues one
# more add per pair (the product kernel's own reference), not counted.
PAIR_F, PAIR_E = 31.0, 2.0
# Scaled HBM bytes of one k_loo_diag<float,5,1,grad> launch at N=500k, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE runs, each scaled by the same counter's
# reading for a 256 MiB copy (profiles/k_loo_diag_f32_5x1_grad_photoz500k.md).
# Set to None whenever that kernel changes, until the counters are re-taken.
DIAG_TRAFFIC_BYTES = 958_886_000
# Shader-clock cycles of one such launch: rocprofv3 --pmc GRBM_COUNT over the
# launch, divided by the 8 XCDs the counter sums over.  Two runs on two boxes
# (3 launches each): 3.996e8 cycles at 2.20 GHz and 3.944e8 at 2.30 GHz, so
# the launch's cycle count holds while the clock, and with it the time,
# varies from box to box.  The ideal cycle count over the mean is the
# roofline fraction at the measured clock.  None whenever that kernel
# changes, until the counter is re-taken.
DIAG_CYCLES = 397_000_000
DIAG_CYCLES_GHZ = "2.20-2.30"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=500_000)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target wall time of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=50.0,
                    help="arrival rate of the short serving stream (0: skip it)")
    ap.add_argument("--serve-duration", type=float, default=20.0,
                    help="seconds of arrivals of the short serving stream")
    ap.add_argument("--no-query", action="store_true", help="skip the density-query secondary")
    ap.add_argument("--trace-steps", type=int, default=0,
                    help="after the timed steps, run this many untimed ascent steps from the "
                         "normal-reference start and report the whole trace of S")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy first (a known-size kernel "
                         "for scaling hardware byte counters)")
    return ap.parse_args()


def host_cpu():
    """(threads the oracle may use, nproc, CPU model): every core this
    process may run on, capped by OMP_NUM_THREADS when the host sets it (a
    multi-GPU host can give each GPU a share of its cores that way)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(avail, int(omp)) if omp.isdigit() and int(omp) > 0 else avail
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return threads, os.cpu_count() or 1, model


def cpu_baseline(x64, y64, h, target_s):
    """The FP64 oracle (unchanged) on a bounded sample: m points i, each
    against all N points j, value and gradient, on every host core this
    process may use."""
    import numpy as np

    import oracle
    threads, nproc, cpu_model = host_cpu()
    n = x64.shape[0]
    rng = np.random.default_rng(123)
    m = 8 * threads
    while True:
        idx = np.sort(rng.choice(n, size=m, replace=False))
        t0 = time.perf_counter()
        oracle.loo(x64, y64, h, idx=idx, grad=True, nthreads=threads)
        dt = time.perf_counter() - t0
        if dt >= 0.25 * target_s or m >= n:
            break
        m = min(n, int(m * max(2.0, 0.5 * target_s / max(dt, 1e-3))))
    rate = m * (n - 1) / dt
    return {"value": rate, "unit": "pair-kernel evals/s", "cores": threads, "kind": "oracle",
            "nproc": nproc, "cpu_model": cpu_model,
            "sample": f"value+gradient for {m} sampled points i, each against all {n - 1} j != i "
                      f"(single-setting FP64 oracle, {threads} threads = the cores this process may "
                      f"use (nproc {nproc}, OMP_NUM_THREADS {os.environ.get('OMP_NUM_THREADS', 'unset')}), "
                      f"{dt:.2f} s wall)"}


# Dense FP32 matrix-core peak of MI355X (FLOP/s, an FMA counted as two).
MFMA_F32_PEAK = 157.3e12


def query_secondary(model, x32, y32, h, q=16384, k=256, reps=3):
    """Density queries (eq. 1) on the same resident training set: q query
    points (training points plus N(0, 0.05^2) noise, seed 7) on a k-point y
    grid, the batch of bench_query.py.  Mean HIP-event time of one call on
    the stream it runs on, and its fraction of the FP32 matrix-core peak for
    the 2 q n k FLOP of the contraction."""
    import numpy as np
    import torch

    n, dx = x32.shape
    rng = np.random.default_rng(7)
    xq = (x32[rng.choice(n, q)] + 0.05 * rng.standard_normal((q, dx))).astype(np.float32)
    ys = y32[:, 0].astype(np.float64)
    yg = np.linspace(ys.min() - 3 * ys.std(), ys.max() + 3 * ys.std(), k).astype(np.float32)
    dev = torch.device("cuda:0")
    xqd = torch.from_numpy(xq).to(dev)
    ygd = torch.from_numpy(yg.reshape(-1, 1)).to(dev)
    stream = torch.cuda.current_stream()
    model.query(xqd, ygd, h, stream=stream)  # warm-up (grows the model's scratch)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        model.query(xqd, ygd, h, stream=stream)
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    t = float(np.mean(ms))
    flops = 2.0 * q * n * k
    return {"workload": f"{q} queries x {k}-point y grid against the same {n} points", "ms": t,
            "queries_per_s": q / (t * 1e-3),
            "roofline": {"bound": "mfma", "achieved": flops / (t * 1e-3) / 1e12, "peak": MFMA_F32_PEAK / 1e12,
                         "unit": "TFLOP/s", "frac": flops / (t * 1e-3) / MFMA_F32_PEAK,
                         "work": "2 q n k FLOP of the contraction; whole call timed"}}


def serve_secondary(rate, duration):
    """The metric's serving half on a short seeded stream: the same requests
    through the one-request-per-launch server and the continuous-batching
    server (grouped job launches, fused query launches); p50/p99 latency,
    throughput and whether every result is bit-identical between the two.
    Stream: Poisson arrivals, 70% density queries (1..4096 points, 256-point
    y grid, with conditional mean and summaries) against 8 resident sets, 30%
    16 x 16 bandwidth-selection jobs with n log-uniform in [1k, 200k]."""
    import copy

    import bench_serve
    import workloads
    from paper_1206_5278_amd.serve import GpuExecutor

    sets = workloads.resident_sets(8, seed=0)
    reqs = bench_serve.build_requests(workloads.serve_stream(rate=rate, duration=duration, seed=5), sets,
                                      seed=5)
    ex = GpuExecutor(sets)
    budget = 96 << 30
    bench_serve.run_mode(ex, copy.deepcopy(reqs[:4]), True, budget, 60.0)  # warm-up
    out = {"rate_req_s": rate, "duration_s": duration, "requests": len(reqs),
           "jobs": sum(r.kind == "job" for r in reqs)}
    results = {}
    for mode, batched in (("plain", False), ("batched", True)):
        rep, results[mode] = bench_serve.run_mode(ex, copy.deepcopy(reqs), batched, budget, 300.0)
        out[mode] = {k: rep[k] for k in ("throughput_req_s", "p50_s", "p99_s", "makespan_s", "completed",
                                         "failed", "unfinished")}
        out[mode]["job_p99_s"] = rep["job"]["p99_s"]
        out[mode]["query_p99_s"] = rep["query"]["p99_s"]
        print(f"bench: serving stream, {mode} mode done", file=sys.stderr, flush=True)
    common = set(results["plain"]) & set(results["batched"])
    out["results_identical_alone_vs_mixed"] = all(results["plain"][k] == results["batched"][k]
                                                  for k in common)
    out["compared"] = len(common)
    for st in ex.sets:
        st["model"].close()
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only; multi-GPU runs are not supported "
              "(the path shards by point ranges with one all-reduce of the totals; not built)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1206_5278_amd as cde
    import workloads

    n = args.n
    x, y = workloads.photoz(n, seed=0)
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    y32 = np.ascontiguousarray(y, dtype=np.float32)
    dev = torch.device("cuda:0")
    model = cde.Model(torch.from_numpy(x32).to(dev), torch.from_numpy(y32).to(dev))
    h0 = cde.normal_reference_bandwidths(x32.astype(np.float64), y32.astype(np.float64))

    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    theta = torch.log(h0.clone()).requires_grad_(True)
    opt = torch.optim.Adam([theta], lr=0.05, betas=(0.9, 0.999))
    stream = torch.cuda.current_stream()
    ev = []

    def step(timed):
        opt.zero_grad()
        if timed:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        s = cde.LooLogLik.apply(theta, model, "cond")
        if timed:
            e1.record(stream)
            ev.append((e0, e1))
        (-s).backward()
        opt.step()
        return float(s.detach())

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    trace = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        trace.append(step(True))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    pairs = float(n) * (n - 1)
    value = pairs / (wall / args.steps)

    # The event pair brackets the pair kernel k_loo_diag (>99.9% of it), the
    # 0.13 ms chunk combine and the few-microsecond block-partial reduction
    # that follow it on the same stream.
    kern_ms = sum(a.elapsed_time(b) for a, b in ev) / len(ev)
    slots = pairs * (PAIR_F + EXP_SLOTS * PAIR_E)
    achieved = slots / (kern_ms * 1e-3) / 1e12
    peak = VALU_PEAK_SLOTS / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tslot/s",
                "frac": achieved / peak,
                "traffic": DIAG_TRAFFIC_BYTES if n == 500_000 else None,
                "kernel": "k_loo_diag<float,5,1,grad>", "kernel_ms": kern_ms,
                "measured_clock": ({"frac": slots / (VALU_PEAK_SLOTS / 2.4e9) / DIAG_CYCLES,
                                    "cycles_per_launch": DIAG_CYCLES, "ghz": DIAG_CYCLES_GHZ,
                                    "source": "rocprofv3 --pmc GRBM_COUNT / 8 XCDs over the launch"}
                                   if n == 500_000 and DIAG_CYCLES else None),
                "work_per_pair": f"F={PAIR_F:g} VALU ops + E={PAIR_E:g} v_exp_f32 x {EXP_SLOTS:g} slots"}

    # Secondary: value-only evaluation (no gradient moments) at the final h.
    h_last = torch.exp(theta.detach()).tolist()
    model.loo_list([h_last])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        model.loo_list([h_last])
    torch.cuda.synchronize()
    vo_ms = 1e3 * (time.perf_counter() - t0) / 3

    trace_run = None
    if args.trace_steps > 0:
        t0 = time.perf_counter()
        st = cde.ascend(model, h0.tolist(), steps=args.trace_steps)
        tr = st["trace"]
        trace_run = {"steps": args.trace_steps, "first": tr[0], "last": tr[-1], "max": max(tr),
                     "argmax_step": int(max(range(len(tr)), key=lambda k: tr[k])),
                     "nondecreasing_steps": int(sum(b >= a for a, b in zip(tr, tr[1:]))),
                     "h_start": h0.tolist(), "h_end": st["h"], "trace": tr,
                     "wall_s": time.perf_counter() - t0}
        print(f"bench: ascent trace of {args.trace_steps} steps done", file=sys.stderr, flush=True)

    query = None
    if not args.no_query:
        try:
            query = query_secondary(model, x32, y32, h0.tolist())
        except Exception as e:  # the headline line is printed regardless
            query = {"error": str(e)}

    serve = None
    if args.serve_rate > 0:
        serve = serve_secondary(args.serve_rate, args.serve_duration)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(x32.astype(np.float64), y32.astype(np.float64), h0.tolist(),
                           args.cpu_seconds)

    out = {
        "metric": "LOO-loglik pair-kernel evals/s at N=500k (value+gradient, diagonal bandwidths)",
        "value": value, "unit": "pair-kernel evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "photoz-shaped gradient ascent (value+gradient per step)", "n": n,
                   "dx": 5, "dy": 1, "bandwidths": "diagonal, 6 parameters",
                   "start": "normal-reference rule", "optimizer": "Adam lr 0.05 on log h",
                   "accumulation": "FP32 kernel values and 32-pair subtile sums, FP64 per-point totals, FP64 log/reduce"},
        "roofline": roofline, "cpu_baseline": cpu,
        "trace_first_last": [trace[0], trace[-1]] if trace else None,
        "secondary": {"value_only_ms": vo_ms, "value_only_pair_evals_per_s": pairs / (vo_ms * 1e-3),
                      "query": query, "serve": serve},
    }
    if trace_run is not None:
        out["ascent"] = trace_run
    print(json.dumps(out))
    model.close()


if __name__ == "__main__":
    main()
