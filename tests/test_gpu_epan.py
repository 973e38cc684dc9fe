"""GPU parity of the Epanechnikov-kernel LOO likelihood (the kernel of the
paper's experiments, Section 4) against the FP64 CPU oracle, through the C
ABI: every shape, both precisions and criteria, ragged and multi-chunk sizes,
bandwidths from "every point diverges" to "no tile is skipped", the grid
call, per-point order (the GPU works in a spatial order and must scatter back)
and run-to-run bits."""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests import parity as P

pytestmark = pytest.mark.gpu

NT = min(16, os.cpu_count() or 1)
DIMS = [(dx, dy) for dx in (1, 2, 3, 4, 5, 6, 7, 8, 16) for dy in (1, 2)]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1206_5278_amd  # noqa: F401


def cde():
    import paper_1206_5278_amd as m
    return m


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def check_points(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin), (int(np.sum(np.isfinite(got) != fin)), "finite masks differ")
    assert np.all(got[~fin] == ref[~fin])
    if fin.any():
        P.assert_points(got[fin], ref[fin])


def check_total(got, ref_points):
    ref = oracle.total(ref_points)
    if not np.isfinite(ref):
        assert got == ref, (got, ref)
    else:
        P.assert_total(got, ref, ref_points)


def run_list(x, y, hs, crit="cond", dtype=torch.float32):
    if dtype == torch.float32:
        xo, yo, xd, yd = P.f32_pair(x, y)
    else:
        xo, yo = np.asarray(x, np.float64), np.asarray(y, np.float64)
        xd, yd = P.to_dev(xo, torch.float64), P.to_dev(yo, torch.float64)
    m = cde().Model(xd, yd)
    tot, pp = m.loo_list(hs, crit, per_point=True, kernel="epanechnikov")
    torch.cuda.synchronize()
    refs = [oracle.loo_epan(xo, yo, m._bw(h), crit, nthreads=NT) for h in hs]
    return tot.cpu().numpy(), pp.cpu().numpy(), refs, m


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("crit", ["cond", "joint"])
def test_epan_photoz_bandwidth_sweep(crit, dtype):
    # From bandwidths at which most points diverge to ones that cover most of
    # the data; 2000 points span 8 tiles with a ragged tail.
    say(f"case: epan photoz n=2000 {crit} {dtype}")
    x, y = workloads.photoz(2000, seed=7)
    sd = np.std(np.concatenate([x, y], axis=1), axis=0)
    hs = [list(f * sd) for f in (0.01, 0.05, 0.2, 0.6, 2.0, 8.0)]
    tot, pp, refs, _ = run_list(x, y, hs, crit, dtype)
    for s, ref in enumerate(refs):
        check_points(pp[s], ref)
        check_total(tot[s], ref)


@pytest.mark.parametrize("dx,dy", DIMS)
def test_epan_all_shapes(dx, dy):
    say(f"case: epan shape dx={dx} dy={dy}")
    v = workloads.gmm_general(700, dx + dy, seed=300 + dx * 10 + dy)
    x, y = v[:, :dx], v[:, dx:]
    sd = np.std(v, axis=0)
    hs = [list(0.8 * sd), list(2.5 * sd)]
    tot, pp, refs, _ = run_list(x, y, hs)
    for s, ref in enumerate(refs):
        check_points(pp[s], ref)
        check_total(tot[s], ref)


@pytest.mark.parametrize("n", [2, 3, 255, 257, 513])
def test_epan_edge_sizes(n):
    say(f"case: epan edge n={n}")
    rng = np.random.default_rng(n + 1)
    x = rng.normal(size=(n, 2))
    y = rng.normal(size=(n, 1))
    tot, pp, refs, _ = run_list(x, y, [[1.5, 1.5, 1.5], [3.0, 3.0, 3.0]])
    for s, ref in enumerate(refs):
        check_points(pp[s], ref)
        check_total(tot[s], ref)


def test_epan_large_multi_chunk_sampled():
    # 60,000 points: many j chunks and skipped tiles; 300 sampled points
    # against the oracle (each against all n-1 others) and the finite mask
    # of all points against per-point oracle values of a second sample.
    say("case: epan gmm n=60000 sampled")
    x, y = workloads.gmm(60_000, seed=9, dx=3)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    h = [0.25, 0.25, 0.25, 0.15]
    tot, pp = m.loo_list([h], "cond", per_point=True, kernel="epanechnikov")
    torch.cuda.synchronize()
    pp = pp.cpu().numpy()[0]
    idx = np.random.default_rng(1).choice(60_000, 300, replace=False)
    ref = oracle.loo_epan(xo, yo, h, "cond", idx=idx, nthreads=NT)
    check_points(pp[idx], ref)
    # the total is the sum of the per-point values (fixed order, FP64)
    fin = np.isfinite(pp)
    if fin.all():
        assert abs(float(tot[0]) - oracle.total(pp)) <= 1e-9 * np.sum(np.abs(pp))
    else:
        assert float(tot[0]) == -np.inf


def test_epan_grid_call_and_nonfinite_count():
    say("case: epan grid 4x3")
    x, y = workloads.gmm(1500, seed=10, dx=2)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    hx, hy = [0.05, 0.3, 1.0, 3.0], [0.02, 0.2, 1.0]
    tot, pp, nonfin = m.loo_grid(hx, hy, "cond", per_point=True, kernel="epanechnikov")
    torch.cuda.synchronize()
    tot, pp = tot.cpu().numpy(), pp.cpu().numpy()
    expect_nonfinite = 0
    for a, ha in enumerate(hx):
        for b, hb in enumerate(hy):
            r = oracle.loo_epan(xo, yo, [ha, hb], "cond", nthreads=NT)
            check_points(pp[a * len(hy) + b], r)
            check_total(tot[a * len(hy) + b], r)
            expect_nonfinite += int(np.sum(~np.isfinite(r)))
    assert int(nonfin.item()) == expect_nonfinite
    assert expect_nonfinite > 0  # the smallest bandwidths diverge


def test_epan_deterministic_and_model_order_independent():
    say("case: epan determinism")
    x, y = workloads.photoz(5000, seed=12)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    sd = np.std(np.concatenate([xo, yo], axis=1), axis=0)
    hs = [list(0.3 * sd), list(1.0 * sd)]
    t1, p1 = m.loo_list(hs, per_point=True, kernel="epanechnikov")
    t2, p2 = m.loo_list(hs, per_point=True, kernel="epanechnikov")
    torch.cuda.synchronize()
    assert torch.equal(t1, t2) and torch.equal(p1, p2)
    # a permuted copy of the data gives the permuted per-point values (the
    # spatial order, not the input order, drives the arithmetic)
    perm = np.random.default_rng(3).permutation(5000)
    m2 = cde().Model(xd[perm].contiguous(), yd[perm].contiguous())
    _, p3 = m2.loo_list(hs, per_point=True, kernel="epanechnikov")
    torch.cuda.synchronize()
    np.testing.assert_allclose(p3.cpu().numpy(), p1.cpu().numpy()[:, perm], rtol=1e-12, atol=1e-12)


def check_density(f, ref):
    # query tolerance; rows with no training x inside the window are 0 on both
    peak = ref.max(axis=1, keepdims=True)
    err = np.abs(f - ref)
    assert np.all(err <= 1e-5 * ref + 1e-7 * peak), float(np.max(err / (1e-5 * ref + 1e-7 * peak + 1e-300)))
    assert np.array_equal(f == 0.0, ref == 0.0), int(np.sum((f == 0.0) != (ref == 0.0)))


@pytest.mark.parametrize("dx,dy,k", [(3, 1, 150), (1, 1, 40), (2, 2, 100), (5, 1, 256), (16, 2, 70)])
def test_epan_query_parity(dx, dy, k):
    # 200 queries (two blocks, ragged), grid widths 64/128/256 per block; a
    # narrow and a wide window (the narrow one leaves some queries with no
    # training x inside, f = 0 there, and most grid points outside every window)
    say(f"case: epan query dx={dx} dy={dy} k={k}")
    v = workloads.gmm_general(3000, dx + dy, seed=600 + 10 * dx + dy)
    x, y = v[:, :dx], v[:, dx:]
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    rng = np.random.default_rng(dx + 7 * dy)
    xq = (xo[rng.choice(3000, 200)] + 0.3 * rng.normal(size=(200, dx))).astype(np.float32).astype(np.float64)
    xq[0] = xo.max(axis=0) + 50.0  # far outside the data: D = 0
    yg = (np.linspace(-1, 1, k)[:, None] * np.ones((1, dy)) * 6.0).astype(np.float32).astype(np.float64)
    sd = np.std(np.concatenate([xo, yo], axis=1), axis=0)
    for f_h in (0.15, 0.8):
        h = list(f_h * sd)
        f = m.query(P.to_dev(xq), P.to_dev(yg), h, kernel="epanechnikov").cpu().numpy()
        ref = oracle.density_epan(xo, yo, h, xq, yg)
        check_density(f, ref)
        assert np.all(f[0] == 0.0)


def test_epan_query_rows_independent_of_batch_and_fp64_rejected():
    say("case: epan query rows alone vs batch")
    from paper_1206_5278_amd import _binding as B
    x, y = workloads.photoz(40_000, seed=3)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    sd = np.std(np.concatenate([xo, yo], axis=1), axis=0)
    h = list(0.2 * sd)
    rng = np.random.default_rng(4)
    xq = (xo[rng.choice(40_000, 1000)] + 0.01).astype(np.float32)
    yg = np.linspace(-0.1, 0.7, 256).astype(np.float32)
    xq_d, yg_d = P.to_dev(xq, torch.float32), P.to_dev(yg, torch.float32)
    full = m.query(xq_d, yg_d, h, kernel="epanechnikov").cpu().numpy()
    for rows in ([0], [999], [5, 500, 998]):
        part = m.query(xq_d[rows].contiguous(), yg_d, h, kernel="epanechnikov").cpu().numpy()
        assert np.array_equal(part, full[rows]), rows
    ref = oracle.density_epan(xo, yo, h, xq[[0, 999]].astype(np.float64), yg.astype(np.float64))
    check_density(full[[0, 999]], ref)
    m64 = cde().Model(P.to_dev(x, torch.float64), P.to_dev(y, torch.float64))
    with pytest.raises(B.CdeError) as e:
        m64.query(P.to_dev(xq[:4].astype(np.float64), torch.float64), P.to_dev(yg.astype(np.float64), torch.float64),
                  h, kernel="epanechnikov")
    assert e.value.status == B.CDE_EUNSUPPORTED


def test_epan_query_narrow_window_skipping():
    # n = 120,000 and h = 0.03 sd: almost every (query block, tile) pair is
    # skipped; some queries lie in empty windows.  Rows alone vs in the batch,
    # and sampled rows against the oracle (zeros exactly where it has zeros).
    say("case: epan query n=120000 h=0.03 sd")
    x, y = workloads.photoz(120_000, seed=5)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    sd = np.std(np.concatenate([xo, yo], axis=1), axis=0)
    h = list(0.03 * sd)
    rng = np.random.default_rng(6)
    xq = (xo[rng.choice(120_000, 2500)] + 0.02 * rng.normal(size=(2500, 5))).astype(np.float32)
    yg = np.linspace(-0.1, 0.7, 200).astype(np.float32)
    xq_d, yg_d = P.to_dev(xq, torch.float32), P.to_dev(yg, torch.float32)
    full = m.query(xq_d, yg_d, h, kernel="epanechnikov").cpu().numpy()
    rows = [0, 1234, 2499]
    part = m.query(xq_d[rows].contiguous(), yg_d, h, kernel="epanechnikov").cpu().numpy()
    assert np.array_equal(part, full[rows])
    ref = oracle.density_epan(xo, yo, h, xq[rows].astype(np.float64), yg.astype(np.float64))
    check_density(full[rows], ref)
    assert np.any(full.max(axis=1) == 0.0) and np.any(full.max(axis=1) > 0.0)

