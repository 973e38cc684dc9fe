"""Grid workloads: time of the scalar-bandwidth grid path.

* tiny    -- N = 2,000, dx = dy = 1, FP64, 8 x 8 grid (launch-bound).
* gmm     -- N = 50,000, dx = 5, dy = 1, FP32, 32 x 32 grid.
* photoz  -- N = 500,000, dx = 5, dy = 1, FP32, 16 x 16 grid (the headline
             data on a scalar grid).
* highdim -- N = 1,000,000, dx = 16, dy = 2, FP32, 16 x 16 grid, with the
             x-distances from FP64 coordinate differences (VALU) and with the
             split-bf16 x3 MFMA cross term.

Pair-kernel evaluations per grid: N (N - 1) G.  Prints one JSON line.  The
errors of these calls against the FP64 oracle (sampled points, subset
totals) are reported by ``python -m tests.fullsize_report --grid``.
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--skip-highdim", action="store_true",
                    help="skip the two large sets (photoz 500k and highdim 1M)")
    ap.add_argument("--highdim-only", action="store_true",
                    help="only the 1M-point 16-D set, with its three x-distance variants")
    ap.add_argument("--variant", choices=("valu_fp64_differences", "valu_fp32_differences",
                                          "mfma_bf16x3_cross_term"), default=None,
                    help="with --highdim-only: run this x-distance variant alone (profiling)")
    args = ap.parse_args()
    import numpy as np
    import torch

    import paper_1206_5278_amd as cde
    import workloads
    from paper_1206_5278_amd import _binding as B
    dev = torch.device("cuda:0")
    out = {"metric": "grid LOO-loglik pair-kernel evals/s"}

    if args.highdim_only:
        highdim(out, cde, workloads, B, np, torch, dev, only=args.variant)
        print(json.dumps(out))
        return

    # tiny, FP64
    x, y = workloads.tiny()
    hx, hy = workloads.WORKLOADS["tiny"]["grid"]
    m = cde.Model(torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev))
    dt, tot, _ = timed_grid(m, hx, hy, 5, B.CDE_XTERM_AUTO)
    out["tiny"] = {"ms": dt * 1e3, "evals_per_s": 2000 * 1999 * 64 / dt,
                   "argmax": int(np.argmax(tot.cpu().numpy()))}
    m.close()
    print(json.dumps({"tiny": out["tiny"]}), file=sys.stderr, flush=True)

    # gmm 50k, 32 x 32
    x, y = workloads.gmm()
    x32, y32 = x.astype(np.float32), y.astype(np.float32)
    hx, hy = workloads.WORKLOADS["gmm"]["grid"]
    m = cde.Model(torch.from_numpy(x32).to(dev), torch.from_numpy(y32).to(dev))
    dt, tot, nf = timed_grid(m, hx, hy, 3, B.CDE_XTERM_AUTO)
    out["gmm"] = {"ms": dt * 1e3, "evals_per_s": 50_000 * 49_999 * 1024 / dt, "nonfinite": int(nf.item())}
    m.close()
    print(json.dumps({"gmm": out["gmm"]}), file=sys.stderr, flush=True)

    if not args.skip_highdim:
        # photoz 500k, 16 x 16
        x, y = workloads.photoz(500_000, seed=0)
        x32, y32 = x.astype(np.float32), y.astype(np.float32)
        hx, hy = workloads.WORKLOADS["photoz"]["grid"]
        m = cde.Model(torch.from_numpy(x32).to(dev), torch.from_numpy(y32).to(dev))
        dt, tot, nf = timed_grid(m, hx, hy, 2, B.CDE_XTERM_AUTO)
        out["photoz"] = {"s": dt, "evals_per_s": 500_000 * 499_999 * 256 / dt, "nonfinite": int(nf.item())}
        m.close()
        print(json.dumps({"photoz": out["photoz"]}), file=sys.stderr, flush=True)

        highdim(out, cde, workloads, B, np, torch, dev)
    print(json.dumps(out))


def highdim(out, cde, workloads, B, np, torch, dev, only=None):
    """The 1M-point 16-D set on its 16 x 16 grid, with each way of forming
    the x-distances (FP64 differences, FP32 differences, split-bf16 x3 MFMA
    cross term) in the same pass structure (or the variant `only`)."""
    hx, hy = workloads.WORKLOADS["highdim"]["grid"]
    x, y = workloads.highdim()
    x32, y32 = x.astype(np.float32), y.astype(np.float32)
    m = cde.Model(torch.from_numpy(x32).to(dev), torch.from_numpy(y32).to(dev))
    res = {}
    for name, xt in (("valu_fp64_differences", B.CDE_XTERM_VALU),
                     ("valu_fp32_differences", B.CDE_XTERM_VALU_F32),
                     ("mfma_bf16x3_cross_term", B.CDE_XTERM_MFMA_BF16X3)):
        if only is not None and name != only:
            continue
        dt, tot, nf = timed_grid(m, hx, hy, 1, xt)
        res[name] = {"s": dt, "evals_per_s": 1e6 * (1e6 - 1) * 256 / dt, "nonfinite": int(nf.item())}
        print(json.dumps({name: res[name]}), file=sys.stderr, flush=True)
    m.close()
    out["highdim"] = res


if __name__ == "__main__":
    main()
