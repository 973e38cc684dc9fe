"""Query-side path on a resident training set: conditional densities on a y
grid (eq. 1, all n training points), the conditional mean E[y|x] and the
per-row summary (mass, mode, narrowest 1 - alpha interval).

Workload: the photoz-shaped set, N = 500,000, dx = 5, dy = 1, FP32 model,
normal-reference bandwidths; a batch of Q = 16,384 query points (training
points plus N(0, 0.05^2) noise) and a 256-point y grid on
[min y - 3 sd, max y + 3 sd].  Each call is timed with HIP events on the
stream it runs on.  Prints one JSON line.  Sampled rows against the FP64
oracle, and the oracle's own rate, are reported by
``python -m tests.fullsize_report --query``.
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
# FP64 VALU peak in lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz.
FP64_PEAK_OPS = 256 * 4 * 16 * 2.4e9
# HBM peak (bytes/s).
HBM_PEAK = 8.0e12


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=500_000)
    ap.add_argument("--q", type=int, default=16384)
    ap.add_argument("--k", type=int, default=256)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--alpha", type=float, default=0.05)
    # accepted and ignored: sampled checks and the oracle's rate are reported
    # by tests/fullsize_report.py
    ap.add_argument("--sample", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--no-cpu-baseline", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()

    import numpy as np
    import torch

    import paper_1206_5278_amd as cde
    import workloads

    n, Q, K = args.n, args.q, args.k
    x, y = workloads.photoz(n, seed=0)
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    y32 = np.ascontiguousarray(y, dtype=np.float32)
    xo, yo = x32.astype(np.float64), y32.astype(np.float64)
    dx, dy = x32.shape[1], y32.shape[1]
    dev = torch.device("cuda:0")
    m = cde.Model(torch.from_numpy(x32).to(dev), torch.from_numpy(y32).to(dev))
    h = cde.normal_reference_bandwidths(xo, yo).tolist()
    rng = np.random.default_rng(7)
    xq = (x32[rng.choice(n, Q)] + 0.05 * rng.standard_normal((Q, dx))).astype(np.float32)
    ys = yo[:, 0]
    yg = np.linspace(ys.min() - 3 * ys.std(), ys.max() + 3 * ys.std(), K).astype(np.float32)
    xqd = torch.from_numpy(xq).to(dev)
    ygd = torch.from_numpy(yg.reshape(-1, 1)).to(dev)
    yg64 = torch.from_numpy(yg.astype(np.float64)).to(dev)
    stream = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ms = []
        out = None
        for _ in range(args.reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            out = fn()
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return out, float(np.mean(ms))

    f, f_ms = timed(lambda: m.query(xqd, ygd, h, stream=stream))
    # the Epanechnikov kernel of Section 4 at one scalar h on sd-scaled data
    sd = np.std(np.concatenate([xo, yo], axis=1), axis=0)
    h_ep = list(0.2 * sd)
    fe, fe_ms = timed(lambda: m.query(xqd, ygd, h_ep, stream=stream, kernel="epanechnikov"))
    mean, mean_ms = timed(lambda: m.conditional_mean(xqd, h, stream=stream))
    summ, summ_ms = timed(lambda: cde.density_summary(f, yg64, args.alpha, stream=stream))
    pairs = float(Q) * n
    q_flops = 2.0 * pairs * K
    # conditional mean, FP64 operations per (query, point) pair at dx = 5,
    # dy = 1: the shift pass (5 differences, 5 squares, 5 FMAs, 1 minimum)
    # and the sum pass (the same 15 for the distance, 1 subtraction, 1 add,
    # 1 FMA), not counting the exponential.
    mean_ops = 2 * 3 * dx + 1 + 1 + 1 + dy
    summ_bytes = Q * K * 8 + K * 8 + Q * 4 * 8

    out = {
        "metric": "conditional-density queries: Q x K grid values over N training points",
        "n": n, "q": Q, "k": K, "dtype": "f32 kernel values and products, f64 shifts and reduce",
        "data": "synthetic (photoz-shaped)",
        "density_query": {"ms": f_ms, "queries_per_s": Q / (f_ms * 1e-3),
                          "roofline": {"bound": "mfma", "achieved": q_flops / (f_ms * 1e-3) / 1e12,
                                       "peak": MFMA_F32_PEAK / 1e12, "unit": "TFLOP/s",
                                       "frac": q_flops / (f_ms * 1e-3) / MFMA_F32_PEAK,
                                       "work": "2 Q N K FLOP of the contraction; whole call timed"}},
        # exact skipping makes the work depend on h and on the data's
        # layout, so no roofline fraction: time and the ratio to the
        # Gaussian call on the same batch
        "density_query_epanechnikov": {"ms": fe_ms, "h": "0.2 sd per dimension",
                                       "queries_per_s": Q / (fe_ms * 1e-3),
                                       "speedup_vs_gaussian": f_ms / fe_ms},
        "conditional_mean": {"ms": mean_ms, "queries_per_s": Q / (mean_ms * 1e-3),
                             "roofline": {"bound": "alu", "achieved": pairs * mean_ops / (mean_ms * 1e-3) / 1e12,
                                          "peak": FP64_PEAK_OPS / 1e12, "unit": "T FP64 lane-op/s",
                                          "frac": pairs * mean_ops / (mean_ms * 1e-3) / FP64_PEAK_OPS,
                                          "work": f"{mean_ops} FP64 ops per (query, point) pair + 1 exp"}},
        "density_summary": {"ms": summ_ms, "rows_per_s": Q / (summ_ms * 1e-3),
                            "roofline": {"bound": "hbm", "achieved": summ_bytes / (summ_ms * 1e-3) / 1e9,
                                         "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                         "frac": summ_bytes / (summ_ms * 1e-3) / HBM_PEAK}},
    }
    print(json.dumps(out))
    m.close()


if __name__ == "__main__":
    main()
