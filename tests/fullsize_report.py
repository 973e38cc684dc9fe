"""Errors against the FP64 oracle at the benchmark sizes, and the oracle's own
speed there, for the workloads of the secondary benchmarks (grid, queries,
cross-validated ISE, Epanechnikov kernel).  The benchmark scripts time the
GPU calls only; this script repeats the same calls on the same seeded inputs
and checks sampled outputs, each computed by the oracle point by point
against the whole training set.  Run from the repository root on a GPU:

    python -m tests.fullsize_report [--grid] [--query] [--ise] [--epan] [--headline] [--highdim]

(no flag: the first four; --headline sums the oracle over all 500,000 points
of the headline workload, about five minutes on 16 threads).  Prints one JSON line per section.  The pass/fail
checks at these sizes live in the ``gpu`` tests; this script reports the
numbers.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NT = min(16, os.cpu_count() or 1)


def rel_point_err(got, ref):
    import numpy as np
    e = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    return {"max": float(e.max()), "median": float(np.median(e))}


def grid_report():
    """Scalar-bandwidth grids: the 2,000-point FP64 set (totals), the 50k
    mixture on 32 x 32 (16 sampled points), the 500k photoz set on 16 x 16
    (16 sampled points) and the 16-D set on 16 x 16 (16
    sampled points of the full 1M set; 256 sampled points of its 20k subset
    and totals of a 5k subset, both x-distance variants)."""
    import numpy as np
    import torch

    import oracle
    import paper_1206_5278_amd as cde
    import workloads
    from paper_1206_5278_amd import _binding as B
    dev = torch.device("cuda:0")
    out = {"section": "grid"}

    x, y = workloads.tiny()
    hx, hy = workloads.WORKLOADS["tiny"]["grid"]
    m = cde.Model(torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev))
    tot = m.loo_grid(hx, hy)[0].cpu().numpy()
    ref = oracle.totals(oracle.loo_grid(x, y, hx, hy, nthreads=NT))
    out["tiny"] = {"max_total_rel_err": float(np.max(np.abs(tot - ref) / np.abs(ref))),
                   "argmax_match": int(np.argmax(tot)) == int(np.argmax(ref))}
    m.close()

    x, y = workloads.gmm()
    x32, y32 = x.astype(np.float32), y.astype(np.float32)
    hx, hy = workloads.WORKLOADS["gmm"]["grid"]
    m = cde.Model(torch.from_numpy(x32).to(dev), torch.from_numpy(y32).to(dev))
    _, pp, nf = m.loo_grid(hx, hy, per_point=True)
    idx = np.sort(np.random.default_rng(3).choice(50_000, 16, replace=False))
    refp = oracle.loo_grid(x32.astype(np.float64), y32.astype(np.float64), hx, hy, idx=idx, nthreads=NT)
    out["gmm"] = {"per_point_err_16_sampled_points": rel_point_err(pp.cpu().numpy()[:, idx], refp),
                  "nonfinite": int(nf.item())}
    del pp
    m.close()

    x, y = workloads.photoz(500_000, seed=0)
    x32, y32 = x.astype(np.float32), y.astype(np.float32)
    hx, hy = workloads.WORKLOADS["photoz"]["grid"]
    m = cde.Model(torch.from_numpy(x32).to(dev), torch.from_numpy(y32).to(dev))
    _, pp, nf = m.loo_grid(hx, hy, per_point=True)
    idx = np.sort(np.random.default_rng(23).choice(500_000, 16, replace=False))
    got = pp[:, torch.from_numpy(idx).to(pp.device)].cpu().numpy()
    del pp
    m.close()
    refp = oracle.loo_grid(x32.astype(np.float64), y32.astype(np.float64), hx, hy, idx=idx, nthreads=NT)
    out["photoz"] = {"per_point_err_16_sampled_points": rel_point_err(got, refp), "nonfinite": int(nf.item())}

    out.update(highdim_report())
    return out


def highdim_report():
    """The 16-D set on its 16 x 16 grid: 16 sampled points of the full 1M set
    (default x-distances), then for each way of forming the x-distances (FP64
    differences, FP32 differences, split-bf16 x3 MFMA cross term) 256 sampled
    points of the 20k subset and the totals of a 5k subset."""
    import numpy as np
    import torch

    import oracle
    import paper_1206_5278_amd as cde
    import workloads
    from paper_1206_5278_amd import _binding as B
    dev = torch.device("cuda:0")
    out = {"section": "highdim"}
    hx, hy = workloads.WORKLOADS["highdim"]["grid"]
    x, y = workloads.highdim()
    # the full 1M-point set: 16 sampled points against all other points
    x32f, y32f = x.astype(np.float32), y.astype(np.float32)
    m = cde.Model(torch.from_numpy(x32f).to(dev), torch.from_numpy(y32f).to(dev))
    _, pp, _ = m.loo_grid(hx, hy, per_point=True)
    idx = np.sort(np.random.default_rng(19).choice(len(x32f), 16, replace=False))
    got = pp[:, torch.from_numpy(idx).to(pp.device)].cpu().numpy()
    del pp
    m.close()
    ref = oracle.loo_grid(x32f.astype(np.float64), y32f.astype(np.float64), hx, hy, idx=idx, nthreads=NT)
    out["highdim_full_1m"] = {"per_point_err_16_sampled_points": rel_point_err(got, ref)}
    xs, ys = workloads.subsample(x, y, 20_000, seed=1)
    xs32, ys32 = xs.astype(np.float32), ys.astype(np.float32)
    xo, yo = xs32.astype(np.float64), ys32.astype(np.float64)
    m = cde.Model(torch.from_numpy(xs32).to(dev), torch.from_numpy(ys32).to(dev))
    idx = np.sort(np.random.default_rng(5).choice(20_000, 256, replace=False))
    refp = oracle.loo_grid(xo, yo, hx, hy, idx=idx, nthreads=NT)
    x5, y5 = workloads.subsample(xs, ys, 5000, seed=2)
    x5, y5 = x5.astype(np.float32), y5.astype(np.float32)
    ref5 = oracle.totals(oracle.loo_grid(x5.astype(np.float64), y5.astype(np.float64), hx, hy, nthreads=NT))
    m5 = cde.Model(torch.from_numpy(x5).to(dev), torch.from_numpy(y5).to(dev))
    res = {}
    for name, xt in (("valu_fp64_differences", B.CDE_XTERM_VALU),
                     ("valu_fp32_differences", B.CDE_XTERM_VALU_F32),
                     ("mfma_bf16x3_cross_term", B.CDE_XTERM_MFMA_BF16X3)):
        _, pp, _ = m.loo_grid(hx, hy, per_point=True, xterm=xt)
        t5 = m5.loo_grid(hx, hy, xterm=xt)[0].cpu().numpy()
        e = np.abs(t5 - ref5) / np.abs(ref5)
        res[name] = {"subset20k_per_point_err_256_sampled": rel_point_err(pp.cpu().numpy()[:, idx], refp),
                     "subset5k_total_rel_err": {"max": float(e.max()), "median": float(np.median(e))}}
    out["highdim"] = res
    m.close()
    m5.close()
    return out


def headline_report():
    """The headline workload in full: photoz N = 500,000, value and gradient
    at the normal-reference bandwidths, against the oracle summed over all
    500,000 points (in 10 slices of 50,000, a progress line after each).
    Tolerances: total 1e-6 relative; gradient per component 1e-4 of
    max(|g*_k|, 1e-2 max_k |g*_k|)."""
    import math

    import numpy as np
    import torch

    import oracle
    import paper_1206_5278_amd as cde
    import workloads
    n = 500_000
    x, y = workloads.photoz(n, seed=0)
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    y32 = np.ascontiguousarray(y, dtype=np.float32)
    xo, yo = x32.astype(np.float64), y32.astype(np.float64)
    m = cde.Model(torch.from_numpy(x32).cuda(), torch.from_numpy(y32).cuda())
    h = cde.normal_reference_bandwidths(xo, yo).tolist()
    total, grad, _ = m.loo_grad(h)
    total, grad = float(total.item()), grad.cpu().numpy()
    m.close()
    ells, dells = [], []
    t0 = time.perf_counter()
    for c in range(10):
        idx = np.arange(c * 50_000, (c + 1) * 50_000)
        ell, dell = oracle.loo(xo, yo, h, idx=idx, grad=True, nthreads=NT)
        ells.append(ell)
        dells.append(dell)
        print(f"oracle slice {c + 1}/10 done ({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    ell = np.concatenate(ells)
    dell = np.concatenate(dells)
    ref = math.fsum(ell.tolist())
    gref = np.array([math.fsum(dell[:, k].tolist()) for k in range(dell.shape[1])])
    gscale = np.maximum(np.abs(gref), 1e-2 * np.abs(gref).max())
    return {
        "section": "headline", "n": n, "h": h,
        "total": total, "total_oracle": ref, "total_rel_err": abs(total - ref) / abs(ref),
        "grad": grad.tolist(), "grad_oracle": gref.tolist(),
        "grad_err_over_scale_max": float(np.max(np.abs(grad - gref) / gscale)),
        "oracle_seconds": time.perf_counter() - t0, "oracle_cores": NT,
    }


def query_report():
    """Queries on the 500k photoz set (16,384 queries, 256-point grid):
    sampled density rows (Gaussian and Epanechnikov), conditional means,
    summaries of every row, and the oracle's density rate on 16 threads."""
    import numpy as np
    import torch

    import oracle
    import paper_1206_5278_amd as cde
    import workloads

    n, Q, K, alpha = 500_000, 16384, 256, 0.05
    x, y = workloads.photoz(n, seed=0)
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    y32 = np.ascontiguousarray(y, dtype=np.float32)
    xo, yo = x32.astype(np.float64), y32.astype(np.float64)
    dx = x32.shape[1]
    dev = torch.device("cuda:0")
    m = cde.Model(torch.from_numpy(x32).to(dev), torch.from_numpy(y32).to(dev))
    h = cde.normal_reference_bandwidths(xo, yo).tolist()
    rng = np.random.default_rng(7)
    xq = (x32[rng.choice(n, Q)] + 0.05 * rng.standard_normal((Q, dx))).astype(np.float32)
    ys = yo[:, 0]
    yg = np.linspace(ys.min() - 3 * ys.std(), ys.max() + 3 * ys.std(), K).astype(np.float32)
    xqd = torch.from_numpy(xq).to(dev)
    ygd = torch.from_numpy(yg.reshape(-1, 1)).to(dev)
    sd = np.std(np.concatenate([xo, yo], axis=1), axis=0)
    h_ep = list(0.2 * sd)
    f = m.query(xqd, ygd, h)
    fe = m.query(xqd, ygd, h_ep, kernel="epanechnikov")
    mean = m.conditional_mean(xqd, h)
    summ = cde.density_summary(f, torch.from_numpy(yg.astype(np.float64)).to(dev), alpha)
    f_np, fe_np, mean_np, summ_np = (t.cpu().numpy() for t in (f, fe, mean, summ))

    idx = np.sort(rng.choice(Q, 16, replace=False))
    xq64 = xq[idx].astype(np.float64)
    f_ref = oracle.density(xo, yo, h, xq64, yg.astype(np.float64), nthreads=NT)
    peak = f_ref.max(axis=1, keepdims=True)
    fe_ref = oracle.density_epan(xo, yo, h_ep, xq64[:4], yg.astype(np.float64))
    pe = fe_ref.max(axis=1, keepdims=True)
    m_ref = oracle.cond_mean(xo, yo, h, xq64)
    s_ref = oracle.density_summary(f_np, yg.astype(np.float64), alpha)
    t0 = time.perf_counter()
    oracle.density(xo, yo, h, xq64[:NT], yg.astype(np.float64), nthreads=NT)
    dt = time.perf_counter() - t0
    m.close()
    return {
        "section": "query", "n": n, "q": Q, "k": K,
        "density_16_sampled_rows": {
            "max_err_rel_to_f_plus_1pct_peak": float(np.max(np.abs(f_np[idx] - f_ref) / (f_ref + 1e-2 * peak))),
            "within_tolerance": bool(np.all(np.abs(f_np[idx] - f_ref) <= 1e-5 * f_ref + 1e-7 * peak))},
        "epanechnikov_4_sampled_rows_within_tolerance":
            bool(np.all(np.abs(fe_np[idx[:4]] - fe_ref) <= 1e-5 * fe_ref + 1e-7 * pe)),
        "conditional_mean_max_abs_err_over_max_abs_y": float(np.max(np.abs(mean_np[idx] - m_ref)) / np.abs(yo).max()),
        "summary_bit_equal_all_rows": bool(np.array_equal(summ_np, s_ref, equal_nan=True)),
        "oracle_density": {"terms_per_s": NT * n * K / dt, "cores": NT,
                           "sample": f"densities of {NT} queries on the {K}-point grid against all {n} points "
                                     f"({dt:.2f} s wall)"},
    }


def ise_report():
    """Cross-validated ISE: T1 and T2 of sampled points against the oracle,
    photoz N = 20,000 (16 points) and the mixture N = 50,000 (4 points)."""
    import numpy as np
    import torch

    import oracle
    import paper_1206_5278_amd as cde
    import workloads
    rows = []
    for name, (x, y), sample in (("photoz N=20000", workloads.photoz(20_000, seed=0), 16),
                                 ("gmm N=50000", workloads.gmm(50_000, seed=0, dx=5), 4)):
        x32 = np.ascontiguousarray(x, dtype=np.float32)
        y32 = np.ascontiguousarray(y, dtype=np.float32)
        xo, yo = x32.astype(np.float64), y32.astype(np.float64)
        n = len(x32)
        m = cde.Model(torch.from_numpy(x32).cuda(), torch.from_numpy(y32).cuda())
        h = cde.normal_reference_bandwidths(xo, yo).tolist()
        _, terms = m.cv_ise(h, terms=True)
        terms = terms.cpu().numpy()
        idx = np.sort(np.random.default_rng(1).choice(n, sample, replace=False))
        t0 = time.perf_counter()
        t1, t2 = oracle.cv_ise(xo, yo, h, idx=idx, nthreads=NT)
        cpu_s = time.perf_counter() - t0
        rows.append({
            "workload": name, "sampled_points": sample,
            "t1_max_rel_err": float(np.max(np.abs(terms[idx, 0] - t1) / t1)),
            "t2_max_err_over_scale": float(np.max(np.abs(terms[idx, 1] - t2) /
                                                  (np.maximum(1.0, np.abs(np.log(t2))) * t2))),
            "oracle": {"products_per_s": sample * float(n - 1) ** 2 / cpu_s, "cores": NT,
                       "sample": f"T1 and T2 of {sample} points ({cpu_s:.2f} s wall)"}})
        m.close()
    return {"section": "ise", "results": rows}


def epan_report():
    """Epanechnikov LOO on photoz N = 500k at h = f sd: 64 sampled points
    per bandwidth, each against all other points."""
    import numpy as np
    import torch

    import oracle
    import paper_1206_5278_amd as cde
    import workloads
    n = 500_000
    x, y = workloads.photoz(n, seed=0)
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    y32 = np.ascontiguousarray(y, dtype=np.float32)
    xo, yo = x32.astype(np.float64), y32.astype(np.float64)
    m = cde.Model(torch.from_numpy(x32).cuda(), torch.from_numpy(y32).cuda())
    sd = np.std(np.concatenate([xo, yo], axis=1), axis=0)
    idx = np.sort(np.random.default_rng(0).choice(n, 64, replace=False))
    rows = []
    for f in (0.02, 0.05, 0.1, 0.2, 0.5):
        h = list(f * sd)
        _, pp = m.loo_list([h], per_point=True, kernel="epanechnikov")
        got = pp.cpu().numpy()[0][idx]
        ref = oracle.loo_epan(xo, yo, h, "cond", idx=idx, nthreads=NT)
        fin = np.isfinite(ref)
        err = float(np.max(np.abs(got[fin] - ref[fin]) / np.maximum(1.0, np.abs(ref[fin])))) if fin.any() else 0.0
        rows.append({"h_over_sd": f, "diverged_in_sample": int(np.sum(~fin)),
                     "finite_mask_matches": bool(np.array_equal(np.isfinite(got), fin)),
                     "max_rel_err_sampled": err})
    m.close()
    return {"section": "epan", "n": n, "sampled_points": 64, "sweep": rows}


def main():
    ap = argparse.ArgumentParser()
    for s in ("grid", "query", "ise", "epan", "headline", "highdim"):
        ap.add_argument(f"--{s}", action="store_true")
    args = ap.parse_args()
    chosen = [s for s in ("grid", "query", "ise", "epan", "headline", "highdim") if getattr(args, s)] or \
        ["grid", "query", "ise", "epan"]
    fns = {"grid": grid_report, "query": query_report, "ise": ise_report, "epan": epan_report,
           "headline": headline_report, "highdim": highdim_report}
    for s in chosen:
        print(f"section: {s}", file=sys.stderr, flush=True)
        print(json.dumps(fns[s]()), flush=True)


if __name__ == "__main__":
    main()
