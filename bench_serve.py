"""Serving benchmark: continuous batching vs one request per launch.

Open-loop Poisson arrivals (default 200 req/s): 70% conditional-density
queries (1..4096 query points, 256-point y grid, returned with the
conditional mean and each row's mass, mode and narrowest 95% interval)
against 8 resident training sets, 30% bandwidth-selection jobs (N log-uniform in [1k, 200k], dx in 1..8,
dy = 1, 16 x 16 grid) on their own data.  Both servers receive the same
seeded request list; the script reports throughput, p50/p99 latency (of the
completed requests and per kind) and whether every result is bit-identical
between the two (each result alone vs in the mix).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import copy
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def build_requests(stream, sets, seed=0, n_cap=None):
    """Materialise workloads.serve_stream descriptors: job data drawn like the
    10-component mixture workload; query points are resident training points
    plus small noise."""
    import numpy as np

    import workloads
    from paper_1206_5278_amd.serve import ServeRequest
    rng = np.random.default_rng(seed)
    g = tuple(workloads.geomspace(0.05, 5.0, 16))
    out = []
    for d in stream:
        if d.kind == "job":
            n = d.n if n_cap is None else min(d.n, n_cap)
            x, y = workloads.gmm(n, seed=d.seed, dx=d.dx)
            out.append(ServeRequest(d.rid, "job", d.t_arrive, x=x.astype(np.float32),
                                    y=y.astype(np.float32), hx=g, hy=g))
        else:
            xs = sets[d.set_id][0]
            idx = rng.integers(0, xs.shape[0], size=d.q)
            xq = xs[idx] + 0.05 * rng.standard_normal((d.q, xs.shape[1]))
            out.append(ServeRequest(d.rid, "query", d.t_arrive, set_id=d.set_id,
                                    xq=xq.astype(np.float32)))
    return out


def job_pairs(r):
    n = r.x.shape[0]
    return float(n) * (n - 1) * len(r.hx) * len(r.hy)


def run_mode(executor, reqs, batched, budget, deadline, progress=None, **sched):
    """One run of `reqs` through a Scheduler; `sched` overrides its settings
    (tick_pairs, ticks_in_flight, small_job_points)."""
    from paper_1206_5278_amd.serve import Scheduler
    s = Scheduler(executor, hbm_budget=budget, max_active=64, batched=batched, **sched)
    s.submit_all(reqs)
    t0 = time.perf_counter()
    s.run(deadline=deadline, progress=progress)
    wall = time.perf_counter() - t0
    rep = s.report(wall)
    done = [r for r in s.completed if r.error is None]
    rep["job_pair_evals_per_s"] = sum(job_pairs(r) for r in done if r.kind == "job") / max(
        rep["makespan_s"], 1e-9)
    rep["wall_s"] = wall
    return rep, {r.rid: digest(r.result) for r in done}


def digest(res) -> str:
    """SHA-256 over a result's arrays in key order: equal digests mean
    bit-identical results (a long stream's raw results would not fit in host
    memory twice)."""
    import hashlib

    import numpy as np
    h = hashlib.sha256()
    for key in sorted(res):
        v = np.ascontiguousarray(np.asarray(res[key]))
        h.update(key.encode())
        h.update(str(v.dtype).encode())
        h.update(str(v.shape).encode())
        h.update(v.tobytes())
    return h.hexdigest()


def same(a, b):
    """Two results (or their digests) are bit-identical."""
    if isinstance(a, str):
        return a == b
    import numpy as np
    if "totals" in a:
        return np.array_equal(a["totals"], b["totals"]) and a["argmax"] == b["argmax"]
    return all(np.array_equal(a[key], b[key], equal_nan=True) for key in ("f", "mean", "summary"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--duration", type=float, default=10.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--stream-seed", type=int, default=None,
                    help="seed of the main stream (default --seed; bench.py's short stream is --seed 0 "
                         "--stream-seed 5 --rate 50 --duration 20)")
    ap.add_argument("--n-cap", type=int, default=None, help="cap job sizes (smoke runs)")
    ap.add_argument("--budget-gb", type=float, default=96.0)
    ap.add_argument("--deadline", type=float, default=600.0)
    ap.add_argument("--no-main", action="store_true", help="run the sweep only")
    ap.add_argument("--sweep", type=str, default="",
                    help="comma-separated extra arrival rates, each run for --sweep-duration")
    ap.add_argument("--sweep-duration", type=float, default=60.0)
    ap.add_argument("--tick-pairs", type=float, default=None,
                    help="batched mode: pair evaluations per large-job range (scheduler default if unset)")
    ap.add_argument("--ticks-in-flight", type=int, default=None,
                    help="batched mode: large-job ranges in flight (scheduler default if unset)")
    ap.add_argument("--progress", type=float, default=30.0,
                    help="seconds between status lines on stderr (0: none)")
    args = ap.parse_args()

    import workloads
    from paper_1206_5278_amd.serve import GpuExecutor

    sets = workloads.resident_sets(8, seed=args.seed)
    sseed = args.seed if args.stream_seed is None else args.stream_seed
    stream = workloads.serve_stream(rate=args.rate, duration=args.duration if not args.no_main else 0.5,
                                    seed=sseed)
    reqs = build_requests(stream, sets, seed=sseed, n_cap=args.n_cap)
    ex = GpuExecutor(sets)
    budget = int(args.budget_gb * (1 << 30))
    sched = {k: v for k, v in (("tick_pairs", args.tick_pairs), ("ticks_in_flight", args.ticks_in_flight))
             if v is not None}
    # warm-up: one small job and one query through every code path
    run_mode(ex, copy.deepcopy(reqs[:4]), True, budget, 60.0)

    out = {"metric": "serving throughput and p50/p99 latency, continuous batching vs one request per launch",
           "data": "synthetic", "dtype": "f32 kernel values, f64 accumulation", "scheduler": sched}
    if not args.no_main:
        res = {}
        results = {}
        for mode, batched in (("plain", False), ("batched", True)):
            rep, o = run_mode(ex, copy.deepcopy(reqs), batched, budget, args.deadline,
                              progress=args.progress or None, **(sched if batched else {}))
            res[mode] = rep
            results[mode] = o
            print(f"{mode}: {json.dumps(rep)}", file=sys.stderr, flush=True)
        common = set(results["plain"]) & set(results["batched"])
        identical = all(same(results["plain"][k], results["batched"][k]) for k in common)
        n_jobs = sum(1 for r in reqs if r.kind == "job")
        offered = sum(job_pairs(r) for r in reqs if r.kind == "job") / args.duration
        out.update({
            "rate_req_s": args.rate, "duration_s": args.duration, "requests": len(reqs), "jobs": n_jobs,
            "queries": len(reqs) - n_jobs, "offered_job_pair_evals_per_s": offered,
            "plain": res["plain"], "batched": res["batched"],
            "throughput_ratio": res["batched"]["throughput_req_s"] / max(res["plain"]["throughput_req_s"], 1e-9),
            "results_identical_alone_vs_mixed": identical, "compared": len(common)})
    if args.sweep:
        sweep = []
        for rate in [float(v) for v in args.sweep.split(",") if v]:
            st = workloads.serve_stream(rate=rate, duration=args.sweep_duration, seed=args.seed + 1)
            rq = build_requests(st, sets, seed=args.seed + 1, n_cap=args.n_cap)
            row = {"rate_req_s": rate, "requests": len(rq), "duration_s": args.sweep_duration}
            outs = {}
            for mode, batched in (("plain", False), ("batched", True)):
                rep, outs[mode] = run_mode(ex, copy.deepcopy(rq), batched, budget, args.deadline,
                                           progress=args.progress or None, **(sched if batched else {}))
                row[mode] = {k: rep[k] for k in ("throughput_req_s", "p50_s", "p99_s", "makespan_s",
                                                 "completed", "failed", "unfinished")}
                row[mode]["job_p50_s"] = rep["job"]["p50_s"]
                row[mode]["job_p99_s"] = rep["job"]["p99_s"]
                row[mode]["query_p50_s"] = rep["query"]["p50_s"]
                row[mode]["query_p99_s"] = rep["query"]["p99_s"]
            common = set(outs["plain"]) & set(outs["batched"])
            row["results_identical_alone_vs_mixed"] = all(outs["plain"][k] == outs["batched"][k]
                                                          for k in common)
            row["compared"] = len(common)
            print(json.dumps(row), file=sys.stderr, flush=True)
            sweep.append(row)
        out["sweep"] = sweep
    print(json.dumps(out))


if __name__ == "__main__":
    main()
