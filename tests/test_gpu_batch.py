"""GPU checks of the grouped launch (``cde_launch_batch``): the grid
criterion (Section 3, eq. 3) over a work list of point ranges of several
models in one launch per pipeline stage.  Totals must be bit-identical to
one ``cde_loo_loglik`` call per model (the same per-point arithmetic) and
within tolerance of the FP64 oracle; ranges of one model may be spread over
several calls, interleaved with other models."""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests import parity as P

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)
HX = workloads.geomspace(0.05, 5.0, 16)
HY = workloads.geomspace(0.05, 5.0, 16)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def cde():
    import paper_1206_5278_amd as m
    return m


def job(n, dx, seed):
    x, y = workloads.gmm(n, seed=seed, dx=dx)
    return P.f32_pair(x, y)


def single_totals(xd, yd, hx=HX, hy=HY, crit="cond"):
    m = cde().Model(xd, yd)
    t, _, nf = m.loo_grid(hx, hy, crit)
    torch.cuda.synchronize()
    out = (t.clone(), int(nf.item()))
    m.close()
    return out


@pytest.mark.parametrize("dx", [3, 1])
def test_batch_of_mixed_jobs_bit_identical_and_vs_oracle(dx):
    sizes = [300, 1000, 2500, 700, 256, 1300, 2048, 555, 4100, 9000]
    print(f"case: grouped launch, {len(sizes)} jobs dx={dx} 16x16", flush=True)
    jobs = [job(n, dx, 60 + k) for k, n in enumerate(sizes)]
    models = [cde().Model(j[2], j[3]) for j in jobs]
    totals = [torch.empty(256, dtype=torch.float64, device="cuda") for _ in jobs]
    nonfin = [torch.full((1,), -1, dtype=torch.int64, device="cuda") for _ in jobs]
    cde().launch_batch([(m, 0, m.n, t, c) for m, t, c in zip(models, totals, nonfin)], HX, HY)
    torch.cuda.synchronize()
    for k, (xo, yo, xd, yd) in enumerate(jobs):
        ref_t, ref_nf = single_totals(xd, yd)
        assert torch.equal(totals[k], ref_t), f"job {k} (n={sizes[k]}) differs from cde_loo_loglik"
        assert int(nonfin[k].item()) == ref_nf == 0
        if sizes[k] <= 2600:
            ell = oracle.loo_grid(xo, yo, HX, HY, nthreads=NT)
            tk = totals[k].cpu().numpy()
            for s in range(0, 256, 17):
                P.assert_total(float(tk[s]), oracle.total(ell[s]), ell[s])


def test_ranges_over_several_calls_interleaved():
    print("case: grouped launch, ranges of 3 jobs over 4 calls", flush=True)
    a, b, c = job(3000, 4, 70), job(700, 4, 71), job(1500, 4, 72)
    ma, mb, mc = (cde().Model(j[2], j[3]) for j in (a, b, c))
    ta, tb, tc = (torch.empty(256, dtype=torch.float64, device="cuda") for _ in range(3))
    lb = cde().launch_batch
    lb([(ma, 0, 1024, None, None), (mb, 0, 256, None, None)], HX, HY)
    lb([(ma, 1024, 2048, None, None), (mb, 256, 700, tb, None), (mc, 0, 512, None, None)], HX, HY)
    lb([(mc, 512, 1500, tc, None)], HX, HY)
    lb([(ma, 2048, 3000, ta, None)], HX, HY)
    torch.cuda.synchronize()
    for (xo, yo, xd, yd), t in ((a, ta), (b, tb), (c, tc)):
        ref, _ = single_totals(xd, yd)
        assert torch.equal(t, ref)
    # a model evaluated by cde_loo_loglik first (shifts already computed)
    # gives the same totals through the grouped launch
    t2 = torch.empty(256, dtype=torch.float64, device="cuda")
    lb([(mb, 0, 700, t2, None)], HX, HY)
    torch.cuda.synchronize()
    assert torch.equal(t2, tb)
    # a smaller grid and the joint criterion
    hx, hy = HX[::3], HY[5:12]
    t3 = torch.empty(len(hx) * len(hy), dtype=torch.float64, device="cuda")
    lb([(mc, 0, 1500, t3, None)], hx, hy, "joint")
    torch.cuda.synchronize()
    ref3, _ = single_totals(c[2], c[3], hx, hy, "joint")
    assert torch.equal(t3, ref3)


def test_batch_argument_errors():
    print("case: grouped launch argument errors", flush=True)
    from paper_1206_5278_amd import _binding as B
    a, b = job(600, 2, 80), job(600, 3, 81)
    ma, mb = cde().Model(a[2], a[3]), cde().Model(b[2], b[3])
    t = torch.empty(256, dtype=torch.float64, device="cuda")
    lb = cde().launch_batch

    def status(fn):
        try:
            fn()
        except B.CdeError as e:
            return e.status
        return 0

    assert status(lambda: lb([(ma, 0, 600, t, None), (mb, 0, 600, t, None)], HX, HY)) == B.CDE_EINVAL
    assert status(lambda: lb([(ma, 256, 600, t, None)], HX, HY)) == B.CDE_EINVAL      # not from 0
    assert status(lambda: lb([(ma, 0, 300, None, None)], HX, HY)) == B.CDE_EINVAL     # i1 not 256k or n
    assert status(lambda: lb([(ma, 0, 600, None, None)], HX, HY)) == B.CDE_EINVAL     # no totals
    assert status(lambda: lb([(ma, 0, 600, t, None)], list(HX) + [6.0], HY)) == B.CDE_EINVAL  # 17 > 16
    assert status(lambda: lb([(ma, 0, 256, None, None)], HX, HY)) == 0
    # mid-evaluation: other calls on the model are refused, and so is a new grid
    assert status(lambda: ma.loo_grid(HX, HY)) == B.CDE_EINVAL
    assert status(lambda: ma.loo_grad([0.5, 0.5, 0.5])) == B.CDE_EINVAL
    assert status(lambda: lb([(ma, 256, 600, t, None)], HX[:8], HY)) == B.CDE_EINVAL
    assert status(lambda: lb([(ma, 256, 600, t, None)], HX, HY)) == 0
    torch.cuda.synchronize()
    ref, _ = single_totals(a[2], a[3])
    assert torch.equal(t, ref)
    assert status(lambda: ma.loo_grad([0.5, 0.5, 0.5])) == 0  # the evaluation is complete


def test_round_points_and_whole_round_ranges():
    """cde_batch_round_points: a positive multiple of 256 points (ranges are
    multiples of 256) and of the device's compute-unit count; a job split at
    one round gives the totals of the whole-job call, bit for bit."""
    print("case: batch round points, n = round + 700, dx 5", flush=True)
    from paper_1206_5278_amd import _binding as B
    lib = B.load()
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    for dx, dy in [(1, 1), (5, 1), (8, 2), (16, 1), (16, 2)]:
        r = lib.cde_batch_round_points(dx, dy)
        assert r > 0 and r % 256 == 0 and r % ncu == 0, (dx, dy, r)
    rnd = lib.cde_batch_round_points(5, 1)
    n = rnd + 700
    x, y, xd, yd = job(n, 5, 90)
    m = cde().Model(xd, yd)
    t = torch.empty(256, dtype=torch.float64, device="cuda")
    cde().launch_batch([(m, 0, rnd, None, None)], HX, HY)
    cde().launch_batch([(m, rnd, n, t, None)], HX, HY)
    torch.cuda.synchronize()
    ref, _ = single_totals(xd, yd)
    assert torch.equal(t, ref)
    m.close()
