"""Grid workloads: time and accuracy of the scalar-bandwidth grid path.

* tiny    -- N = 2,000, dx = dy = 1, FP64, 8 x 8 grid (launch-bound; parity only).
* gmm     -- N = 50,000, dx = 5, dy = 1, FP32, 32 x 32 grid.
* highdim -- N = 1,000,000, dx = 16, dy = 2, FP32, 16 x 16 grid, with the
             x-distances from FP64 coordinate differences (VALU) and with the
             split-bf16 x3 MFMA cross term; error of both against the FP64
             oracle on the 20k-point subset (sampled points against all 20k
             points, and full totals on a 5k-point subset).

Pair-kernel evaluations per grid: N (N - 1) G.  Prints one JSON line.
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


def timed_grid(model, hx, hy, reps, xterm):
    import torch
    tot, _, nf = model.loo_grid(hx, hy, xterm=xterm)  # first call: neighbour shifts
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        tot, _, nf = model.loo_grid(hx, hy, xterm=xterm)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, tot, nf


def rel_point_err(got, ref):
    import numpy as np
    e = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    return {"max": float(e.max()), "median": float(np.median(e))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--skip-highdim", action="store_true")
    args = ap.parse_args()
    import numpy as np
    import torch

    import oracle
    import paper_1206_5278_amd as cde
    import workloads
    from paper_1206_5278_amd import _binding as B
    nt = min(16, os.cpu_count() or 1)
    dev = torch.device("cuda:0")
    out = {"metric": "grid LOO-loglik pair-kernel evals/s and error vs the FP64 oracle"}

    # tiny, FP64
    x, y = workloads.tiny()
    hx, hy = workloads.WORKLOADS["tiny"]["grid"]
    m = cde.Model(torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev))
    dt, tot, _ = timed_grid(m, hx, hy, 5, B.CDE_XTERM_AUTO)
    ref = oracle.totals(oracle.loo_grid(x, y, hx, hy, nthreads=nt))
    out["tiny"] = {"ms": dt * 1e3, "evals_per_s": 2000 * 1999 * 64 / dt,
                   "max_total_rel_err": float(np.max(np.abs(tot.cpu().numpy() - ref) / np.abs(ref))),
                   "argmax_match": int(np.argmax(tot.cpu().numpy())) == int(np.argmax(ref))}
    print(json.dumps({"tiny": out["tiny"]}), file=sys.stderr, flush=True)

    # gmm 50k, 32 x 32
    x, y = workloads.gmm()
    x32, y32 = x.astype(np.float32), y.astype(np.float32)
    hx, hy = workloads.WORKLOADS["gmm"]["grid"]
    m = cde.Model(torch.from_numpy(x32).to(dev), torch.from_numpy(y32).to(dev))
    dt, tot, nf = timed_grid(m, hx, hy, 3, B.CDE_XTERM_AUTO)
    _, pp, _ = m.loo_grid(hx, hy, per_point=True)
    idx = np.sort(np.random.default_rng(3).choice(50_000, 16, replace=False))
    refp = oracle.loo_grid(x32.astype(np.float64), y32.astype(np.float64), hx, hy, idx=idx, nthreads=nt)
    out["gmm"] = {"ms": dt * 1e3, "evals_per_s": 50_000 * 49_999 * 1024 / dt,
                  "per_point_err_16_sampled_points": rel_point_err(pp.cpu().numpy()[:, idx], refp),
                  "nonfinite": int(nf.item())}
    del pp
    print(json.dumps({"gmm": out["gmm"]}), file=sys.stderr, flush=True)

    if not args.skip_highdim:
        hx, hy = workloads.WORKLOADS["highdim"]["grid"]
        x, y = workloads.highdim()
        x32, y32 = x.astype(np.float32), y.astype(np.float32)
        m = cde.Model(torch.from_numpy(x32).to(dev), torch.from_numpy(y32).to(dev))
        res = {}
        for name, xt in (("valu_fp64_differences", B.CDE_XTERM_VALU),
                         ("mfma_bf16x3_cross_term", B.CDE_XTERM_MFMA_BF16X3)):
            dt, tot, nf = timed_grid(m, hx, hy, 1, xt)
            res[name] = {"s": dt, "evals_per_s": 1e6 * (1e6 - 1) * 256 / dt, "nonfinite": int(nf.item())}
            print(json.dumps({name: res[name]}), file=sys.stderr, flush=True)
        m.close()
        # errors on the 20k-point subset
        xs, ys = workloads.subsample(x, y, 20_000, seed=1)
        xs32, ys32 = xs.astype(np.float32), ys.astype(np.float32)
        xo, yo = xs32.astype(np.float64), ys32.astype(np.float64)
        m = cde.Model(torch.from_numpy(xs32).to(dev), torch.from_numpy(ys32).to(dev))
        idx = np.sort(np.random.default_rng(5).choice(20_000, 256, replace=False))
        refp = oracle.loo_grid(xo, yo, hx, hy, idx=idx, nthreads=nt)
        for name, xt in (("valu_fp64_differences", B.CDE_XTERM_VALU),
                         ("mfma_bf16x3_cross_term", B.CDE_XTERM_MFMA_BF16X3)):
            _, pp, _ = m.loo_grid(hx, hy, per_point=True, xterm=xt)
            res[name]["subset20k_per_point_err_256_sampled"] = rel_point_err(pp.cpu().numpy()[:, idx], refp)
        x5, y5 = workloads.subsample(xs, ys, 5000, seed=2)
        x5, y5 = x5.astype(np.float32), y5.astype(np.float32)
        ref5 = oracle.totals(oracle.loo_grid(x5.astype(np.float64), y5.astype(np.float64), hx, hy,
                                             nthreads=nt))
        m5 = cde.Model(torch.from_numpy(x5).to(dev), torch.from_numpy(y5).to(dev))
        for name, xt in (("valu_fp64_differences", B.CDE_XTERM_VALU),
                         ("mfma_bf16x3_cross_term", B.CDE_XTERM_MFMA_BF16X3)):
            t5, _, _ = m5.loo_grid(hx, hy, xterm=xt)
            e = np.abs(t5.cpu().numpy() - ref5) / np.abs(ref5)
            res[name]["subset5k_total_rel_err"] = {"max": float(e.max()), "median": float(np.median(e))}
        out["highdim"] = res
    print(json.dumps(out))


if __name__ == "__main__":
    main()
