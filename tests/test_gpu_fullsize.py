"""Parity at the benchmark sizes, in the launch configuration the benchmark
times: sampled per-point values against the oracle computed point by point
(each sampled i against all N-1 points j), plus properties that hold at any
size.  Also the gradient workload's 5k-point subsample checks (oracle
gradient, finite differences) and the exactness of ascent checkpoints."""
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


def cde():
    import paper_1206_5278_amd as m
    return m


@pytest.fixture(scope="module")
def photoz_full():
    x, y = workloads.photoz(500_000, seed=0)
    xo, yo, xd, yd = P.f32_pair(x, y)
    return xo, yo, cde().Model(xd, yd)


def test_photoz_500k_sampled_points_value_and_grad_call(photoz_full):
    print("case: photoz n=500000 value+grad, 96 sampled points", flush=True)
    xo, yo, m = photoz_full
    h0 = cde().normal_reference_bandwidths(xo, yo).tolist()
    for h in (h0, [0.03, 0.025, 0.03, 0.035, 0.04, 0.012]):
        total, grad, pp = m.loo_grad(h, per_point=True)
        pp = pp.cpu().numpy()
        assert np.all(np.isfinite(pp))
        idx = np.sort(np.random.default_rng(7).choice(500_000, 96, replace=False))
        # include the points with the largest and smallest l_i: the outliers
        idx = np.unique(np.concatenate([idx, [int(np.argmin(pp)), int(np.argmax(pp))]]))
        ref = oracle.loo(xo, yo, h, idx=idx, nthreads=NT)
        P.assert_points(pp[idx], ref)
        # the total is the fixed-order sum of the per-point values
        assert abs(float(total.item()) - float(np.sum(pp))) <= 1e-10 * abs(float(total.item()))
        assert np.all(np.isfinite(grad.cpu().numpy()))


def test_photoz_500k_query_batch_sampled_rows(photoz_full):
    # The density-query batch the benchmarks time (bench_query.py and
    # bench.py's secondary figure): 16,384 queries on a 256-point y grid
    # against all 500,000 points, in one call (8 slices of 2,048 queries).
    # 8 sampled rows against the oracle (each over all points), and rows
    # alone equal to the same rows in the batch.
    print("case: photoz n=500000 query batch q=16384 k=256, 8 sampled rows", flush=True)
    xo, yo, m = photoz_full
    n, dx = xo.shape
    h = cde().normal_reference_bandwidths(xo, yo).tolist()
    rng = np.random.default_rng(7)
    xq = (xo[rng.choice(n, 16384)].astype(np.float32)
          + 0.05 * rng.standard_normal((16384, dx))).astype(np.float32)
    ys = yo[:, 0]
    yg = np.linspace(ys.min() - 3 * ys.std(), ys.max() + 3 * ys.std(), 256).astype(np.float32)
    xqd, ygd = P.to_dev(xq, torch.float32), P.to_dev(yg.reshape(-1, 1), torch.float32)
    f = m.query(xqd, ygd, h).cpu().numpy()
    assert np.all(np.isfinite(f)) and np.all(f >= 0)
    rows = np.sort(np.random.default_rng(5).choice(16384, 8, replace=False))
    ref = oracle.density(xo, yo, h, xq[rows].astype(np.float64), yg.astype(np.float64), nthreads=NT)
    peak = ref.max(axis=1, keepdims=True)
    err = np.abs(f[rows] - ref)
    assert np.all(err <= 1e-5 * ref + 1e-7 * peak), float(np.max(err / (1e-5 * ref + 1e-7 * peak)))
    part = m.query(xqd[rows[:2].tolist()].contiguous(), ygd, h).cpu().numpy()
    assert np.array_equal(part, f[rows[:2]])


def test_photoz_500k_epanechnikov_sampled_points(photoz_full):
    # The Epanechnikov LOO pass in the configuration bench_epan.py times
    # (photoz N = 500,000, h = f sd per dimension, exact tile skipping over
    # the model's spatial order): 32 sampled points per bandwidth against the
    # oracle over all other points, at 0.2 sd, where some points have no
    # neighbour in their window (l_i = -inf, so the total is -inf), and at
    # 32 sd, the smallest multiple with a finite total.
    print("case: photoz n=500000 Epanechnikov LOO, 32 sampled points at 0.2 and 32 sd", flush=True)
    xo, yo, m = photoz_full
    sd = np.std(np.concatenate([xo, yo], axis=1), axis=0)
    idx = np.sort(np.random.default_rng(2).choice(len(xo), 32, replace=False))
    for f in (0.2, 32.0):
        h = list(f * sd)
        tot, pp = m.loo_list([h], per_point=True, kernel="epanechnikov")
        got = pp.cpu().numpy()[0]
        ref = oracle.loo_epan(xo, yo, h, "cond", idx=idx, nthreads=NT)
        fin = np.isfinite(ref)
        assert np.array_equal(np.isfinite(got[idx]), fin), f
        assert np.all(got[idx][~fin] == ref[~fin])
        if fin.any():
            P.assert_points(got[idx][fin], ref[fin])
        if np.isfinite(got).all():
            assert abs(float(tot[0]) - float(np.sum(got))) <= 1e-9 * float(np.sum(np.abs(got)))
        else:
            assert float(tot[0]) == -np.inf


def test_photoz_20k_cv_ise_sampled_points():
    # The cross-validated ISE in the configuration bench_ise.py times
    # (photoz N = 20,000, normal-reference bandwidths): T1 and T2 of 8
    # sampled points against the oracle, each a double sum over all points,
    # and the means against the returned terms.
    print("case: photoz n=20000 cv_ise, 8 sampled points", flush=True)
    x, y = workloads.photoz(20_000, seed=0)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    h = cde().normal_reference_bandwidths(xo, yo).tolist()
    out, terms = m.cv_ise(h, terms=True)
    out, terms = out.cpu().numpy(), terms.cpu().numpy()
    idx = np.sort(np.random.default_rng(1).choice(20_000, 8, replace=False))
    t1, t2 = oracle.cv_ise(xo, yo, h, idx=idx, nthreads=NT)
    assert np.all(np.abs(terms[idx, 0] - t1) <= 1e-5 * t1)
    assert np.all(np.abs(terms[idx, 1] - t2) <= 1e-5 * np.maximum(1.0, np.abs(np.log(t2))) * t2)
    np.testing.assert_allclose(out[1], terms[:, 0].mean(), rtol=1e-12)
    np.testing.assert_allclose(out[2], terms[:, 1].mean(), rtol=1e-12)
    m.close()


def test_photoz_5k_subsample_gradient_vs_oracle_and_fd():
    print("case: photoz 5k subsample gradient", flush=True)
    x, y = workloads.photoz(500_000, seed=0)
    xs, ys = workloads.subsample(x, y, 5000, seed=1)
    xo, yo, xd, yd = P.f32_pair(xs, ys)
    m = cde().Model(xd, yd)
    h = cde().normal_reference_bandwidths(xo, yo).numpy()
    total, grad, pp = m.loo_grad(h.tolist(), per_point=True)
    ell, dell = oracle.loo(xo, yo, h, grad=True, nthreads=NT)
    P.assert_points(pp.cpu().numpy(), ell)
    P.assert_total(float(total.item()), oracle.total(ell), ell)
    g = grad.cpu().numpy()
    rg = dell.sum(axis=0)
    P.assert_grad(g, rg)
    # Central differences, step 1e-4 relative, of the FP64 oracle (its own
    # truncation error is ~1e-8 relative) agree with the GPU adjoint.
    fd = np.empty(6)
    for k in range(6):
        d = 1e-4 * h[k]
        hp, hm = h.copy(), h.copy()
        hp[k] += d
        hm[k] -= d
        fd[k] = (oracle.total(oracle.loo(xo, yo, hp, nthreads=NT)) -
                 oracle.total(oracle.loo(xo, yo, hm, nthreads=NT))) / (2 * d)
    P.assert_grad(g, fd)
    # The same 12 finite-difference points evaluated on the GPU in one list
    # call: a loose sanity check (FP32 noise / 2e-4 dominates).
    hs = []
    for k in range(6):
        for sgn in (1, -1):
            hh = h.copy()
            hh[k] += sgn * 1e-4 * h[k]
            hs.append(hh.tolist())
    tl, _ = m.loo_list(hs)
    tl = tl.cpu().numpy()
    gfd = np.array([(tl[2 * k] - tl[2 * k + 1]) / (2e-4 * h[k]) for k in range(6)])
    assert np.all(np.abs(gfd - g) <= 2e-2 * np.max(np.abs(g)))


def test_gmm_50k_32x32_grid_sampled_points():
    print("case: gmm n=50000 32x32 grid, 8 sampled points", flush=True)
    cfg = workloads.WORKLOADS["gmm"]
    x, y = workloads.gmm()
    hx, hy = cfg["grid"]
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    tot, pp, nonfin = m.loo_grid(hx, hy, per_point=True)
    assert int(nonfin.item()) == 0
    pp = pp.cpu().numpy()
    idx = np.sort(np.random.default_rng(3).choice(50_000, 8, replace=False))
    ref = oracle.loo_grid(xo, yo, hx, hy, idx=idx, nthreads=NT)
    P.assert_points(pp[:, idx], ref)
    t = tot.cpu().numpy()
    np.testing.assert_allclose(t, pp.sum(axis=1), rtol=1e-10)


def test_gmm_300k_16x16_grid_sampled_points():
    # Above 2^18 points the FP64 rerun of flagged points runs 8 points per
    # wave (2 below): 48 sampled points, of which a few are expected to have
    # a flagged cell, each checked against all other 299,999 points.
    print("case: gmm n=300000 16x16 grid, 48 sampled points", flush=True)
    x, y = workloads.gmm(300_000, seed=4, dx=5)
    hx = workloads.geomspace(0.05, 5.0, 16)
    hy = workloads.geomspace(0.05, 5.0, 16)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    tot, pp, nonfin = m.loo_grid(hx, hy, per_point=True)
    assert int(nonfin.item()) == 0
    pp = pp.cpu().numpy()
    idx = np.sort(np.random.default_rng(11).choice(300_000, 48, replace=False))
    ref = oracle.loo_grid(xo, yo, hx, hy, idx=idx, nthreads=NT)
    P.assert_points(pp[:, idx], ref)
    np.testing.assert_allclose(tot.cpu().numpy(), pp.sum(axis=1), rtol=1e-10)
    m.close()


def test_highdim_1m_16x16_grid_sampled_points():
    # The 1,000,000-point 16-D set on its 16 x 16 grid, in the default
    # configuration the benchmark times (FP32 pass with FP64-difference
    # distances, FP64 rerun of flagged points): 16 sampled points, each
    # checked against the oracle over all other 999,999 points.
    print("case: highdim n=1000000 16x16 grid, 16 sampled points", flush=True)
    x, y = workloads.highdim()
    hx, hy = workloads.WORKLOADS["highdim"]["grid"]
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    tot, pp, nonfin = m.loo_grid(hx, hy, per_point=True)
    assert int(nonfin.item()) == 0
    idx = np.sort(np.random.default_rng(19).choice(len(xo), 16, replace=False))
    got = pp[:, torch.from_numpy(idx).to(pp.device)].cpu().numpy()
    np.testing.assert_allclose(tot.cpu().numpy(), pp.sum(dim=1).cpu().numpy(), rtol=1e-10)
    del pp
    m.close()
    ref = oracle.loo_grid(xo, yo, hx, hy, idx=idx, nthreads=NT)
    P.assert_points(got, ref)


def test_ascend_checkpoint_resume_is_exact(tmp_path):
    print("case: ascend checkpoint/resume", flush=True)
    x, y = workloads.photoz(3000, seed=9)
    _, _, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    h0 = cde().normal_reference_bandwidths(x.astype(np.float32), y.astype(np.float32))
    full = cde().ascend(m, h0, steps=6)
    ck = str(tmp_path / "ck.json")
    cde().ascend(m, h0, steps=3, checkpoint=ck)
    import json
    resumed = cde().ascend(m, h0, steps=6, resume=json.load(open(ck)))
    assert resumed["trace"] == full["trace"]
    assert resumed["theta"] == full["theta"]
    # ascent increases the criterion from the normal-reference start
    assert full["trace"][-1] > full["trace"][0]
