"""GPU serving: every request's result is bit-identical alone (one request
per launch) and in the mix (continuous batching with fused query launches and
overlapping jobs), and matches the FP64 oracle."""
import copy
import os

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests import parity as P

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("tick_pairs,small_points", [(1e12, 16384), (3e8, 600)])
def test_serve_alone_vs_mixed_identical_and_oracle(tick_pairs, small_points):
    # (3e8, 600): every job above 600 points runs as ranges over several
    # grouped launches of the large-job lane
    print(f"case: serve small stream, plain vs batched, tick {tick_pairs:g} small {small_points}",
          flush=True)
    import bench_serve
    from paper_1206_5278_amd.serve import GpuExecutor, Scheduler
    sets = [workloads.gmm(n, seed=40 + k, dx=dx) for k, (n, dx) in
            enumerate([(1500, 2), (700, 5), (2500, 1)])]
    stream = workloads.serve_stream(rate=400.0, duration=0.25, seed=3, n_hi=3000, q_max=300,
                                    n_sets=3)
    reqs = bench_serve.build_requests(stream, sets, seed=3)
    assert sum(r.kind == "job" for r in reqs) >= 5 and sum(r.kind == "query" for r in reqs) >= 10
    ex = GpuExecutor(sets, grid_points=64)
    out = {}
    for batched in (False, True):
        s = Scheduler(ex, hbm_budget=8 << 30, batched=batched, tick_pairs=tick_pairs,
                      small_job_points=small_points)
        rs = copy.deepcopy(reqs)
        s.submit_all(rs)
        s.run(deadline=120.0)
        assert all(r.error is None for r in s.completed)
        assert len(s.completed) == len(reqs)
        out[batched] = {r.rid: r.result for r in s.completed}
    for rid in out[False]:
        a, b = out[False][rid], out[True][rid]
        if "totals" in a:
            assert np.array_equal(a["totals"], b["totals"]) and a["argmax"] == b["argmax"]
        else:
            for key in ("f", "mean", "summary"):
                assert np.array_equal(a[key], b[key], equal_nan=True), key
    # spot-check against the oracle: one job (per-setting totals) and one query
    job = next(r for r in reqs if r.kind == "job")
    ref = oracle.totals(oracle.loo_grid(job.x.astype(np.float64), job.y.astype(np.float64),
                                        job.hx, job.hy, nthreads=NT))
    got = out[True][job.rid]["totals"].ravel()
    for k in range(ref.size):
        assert abs(got[k] - ref[k]) <= 1e-6 * abs(ref[k])
    q = next(r for r in reqs if r.kind == "query")
    st = ex.sets[q.set_id]
    xs, ys = sets[q.set_id]
    f_ref = oracle.density(xs.astype(np.float32).astype(np.float64),
                           ys.astype(np.float32).astype(np.float64), st["h"],
                           q.xq.astype(np.float64), st["ygrid"].cpu().numpy().astype(np.float64),
                           nthreads=NT)
    f = out[True][q.rid]["f"]
    peak = f_ref.max(axis=1, keepdims=True)
    assert np.all(np.abs(f - f_ref) <= 1e-5 * f_ref + 1e-7 * peak)
    # the products returned with it
    xs64, ys64 = xs.astype(np.float32).astype(np.float64), ys.astype(np.float32).astype(np.float64)
    m_ref = oracle.cond_mean(xs64, ys64, st["h"], q.xq.astype(np.float32).astype(np.float64))
    assert np.all(np.abs(out[True][q.rid]["mean"] - m_ref) <= 1e-12 * np.abs(ys64).max())
    s_ref = oracle.density_summary(f, st["ygrid64"].cpu().numpy(), 0.05)
    assert np.array_equal(out[True][q.rid]["summary"], s_ref, equal_nan=True)
