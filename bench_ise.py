"""Exact cross-validated ISE (Section 3, eq. 2) on the matrix cores.

Workloads: the photoz-shaped set at N = 20,000 (dx = 5, dy = 1, the size of
the paper's larger SDSS sample) and the 10-component mixture at N = 50,000
(dx = 5, dy = 1), normal-reference bandwidths.  One evaluation is
N (N - 1)^2 x-weighted y-convolution products (the double sum over j, l != i
for every i) plus the exact LOO pass for the second term.  Each call is
timed with HIP events on the stream it runs on; sampled points are checked
against the FP64 oracle; the oracle is timed on the same sample.  Prints one
JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Dense FP32 matrix-core peak of MI355X (FLOP/s, an FMA counted as two).
MFMA_F32_PEAK = 157.3e12


def run(name, x, y, reps, sample, threads):
    import numpy as np
    import torch

    import oracle
    import paper_1206_5278_amd as cde

    x32 = np.ascontiguousarray(x, dtype=np.float32)
    y32 = np.ascontiguousarray(y, dtype=np.float32)
    xo, yo = x32.astype(np.float64), y32.astype(np.float64)
    n = len(x32)
    m = cde.Model(torch.from_numpy(x32).cuda(), torch.from_numpy(y32).cuda())
    h = cde.normal_reference_bandwidths(xo, yo).tolist()
    stream = torch.cuda.current_stream()
    out, terms = m.cv_ise(h, terms=True, stream=stream)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        out = m.cv_ise(h, stream=stream)
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    call_ms = float(np.mean(ms))
    out, terms = out.cpu().numpy(), terms.cpu().numpy()
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(n, sample, replace=False))
    t0 = time.perf_counter()
    t1, t2 = oracle.cv_ise(xo, yo, h, idx=idx, nthreads=threads)
    cpu_s = time.perf_counter() - t0
    e1 = float(np.max(np.abs(terms[idx, 0] - t1) / t1))
    e2 = float(np.max(np.abs(terms[idx, 1] - t2) / (np.maximum(1.0, np.abs(np.log(t2))) * t2)))
    flops = 2.0 * n * float(n - 1) ** 2
    m.close()
    return {
        "workload": name, "n": n, "ms": call_ms, "ise": float(out[0]), "mean_t1": float(out[1]),
        "mean_t2": float(out[2]),
        "products_per_s": n * float(n - 1) ** 2 / (call_ms * 1e-3),
        "roofline": {"bound": "mfma", "achieved": flops / (call_ms * 1e-3) / 1e12,
                     "peak": MFMA_F32_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": flops / (call_ms * 1e-3) / MFMA_F32_PEAK,
                     "work": "2 N (N-1)^2 FLOP of the double sum; whole call timed"},
        "sampled_points": sample, "t1_max_rel_err": e1, "t2_max_err_over_scale": e2,
        "cpu_baseline": {"value": sample * float(n - 1) ** 2 / cpu_s, "unit": "products/s",
                         "cores": threads, "kind": "oracle",
                         "sample": f"T1 and T2 of {sample} points ({cpu_s:.2f} s wall)"},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--sample", type=int, default=16)
    ap.add_argument("--skip-50k", action="store_true")
    args = ap.parse_args()
    import workloads
    threads = min(16, os.cpu_count() or 1)
    rows = [run("photoz N=20000", *workloads.photoz(20_000, seed=0), args.reps, args.sample, threads)]
    if not args.skip_50k:
        rows.append(run("gmm N=50000", *workloads.gmm(50_000, seed=0, dx=5), args.reps,
                        max(4, args.sample // 4), threads))
    print(json.dumps({"metric": "exact cross-validated ISE: x-weighted y-convolution products per second",
                      "dtype": "f32 kernel values and products, f64 folds and totals",
                      "data": "synthetic", "results": rows}))


if __name__ == "__main__":
    main()
