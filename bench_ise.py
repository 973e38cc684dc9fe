"""Exact cross-validated ISE (Section 3, eq. 2) on the matrix cores.

Workloads: the photoz-shaped set at N = 20,000 (dx = 5, dy = 1, the size of
the paper's larger SDSS sample) and the 10-component mixture at N = 50,000
(dx = 5, dy = 1), normal-reference bandwidths.  One evaluation is
N (N - 1)^2 x-weighted y-convolution products (the double sum over j, l != i
for every i) plus the exact LOO pass for the second term.  Each call is
timed with HIP events on the stream it runs on.  Prints one JSON line.
Sampled points against the FP64 oracle, and the oracle's own rate, are
reported by ``python -m tests.fullsize_report --ise``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Dense FP32 matrix-core peak of MI355X (FLOP/s, an FMA counted as two).
MFMA_F32_PEAK = 157.3e12


def run(name, x, y, reps):
    import numpy as np
    import torch

    import paper_1206_5278_amd as cde

    x32 = np.ascontiguousarray(x, dtype=np.float32)
    y32 = np.ascontiguousarray(y, dtype=np.float32)
    xo, yo = x32.astype(np.float64), y32.astype(np.float64)
    n = len(x32)
    m = cde.Model(torch.from_numpy(x32).cuda(), torch.from_numpy(y32).cuda())
    h = cde.normal_reference_bandwidths(xo, yo).tolist()
    stream = torch.cuda.current_stream()
    out = m.cv_ise(h, stream=stream)
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
    out = out.cpu().numpy()
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
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--skip-50k", action="store_true")
    # accepted and ignored: sampled checks are reported by tests/fullsize_report.py
    ap.add_argument("--sample", type=int, default=0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    import workloads
    rows = [run("photoz N=20000", *workloads.photoz(20_000, seed=0), args.reps)]
    if not args.skip_50k:
        rows.append(run("gmm N=50000", *workloads.gmm(50_000, seed=0, dx=5), args.reps))
    print(json.dumps({"metric": "exact cross-validated ISE: x-weighted y-convolution products per second",
                      "dtype": "f32 kernel values and products, f64 folds and totals",
                      "data": "synthetic", "results": rows}))


if __name__ == "__main__":
    main()
