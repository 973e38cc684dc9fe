"""GPU parity of the cross-validated ISE (Section 3, eq. 2) against the FP64
oracle, through the C ABI: per-point terms T1_i (the O(n^2)-per-point double
sum on the matrix cores) and T2_i, the totals, ragged row / column / j
blocks, several FP64 fold segments, tiny and degenerate sets, and the
argument checks.

Tolerances: T1_i is a sum of positive FP32 kernel products with FP32 panel
sums folded into FP64 every 64 panels, |T1 - T1*| <= 1e-5 T1*; T2_i =
exp(l_i) inherits the per-point LOO tolerance, |T2 - T2*| <= 1e-5 max(1,
|log T2*|) T2*; the ISE total is held to 1e-6 of sum_i (T1_i + 2 T2_i) / n
(the total is a difference of two means and may be near zero)."""
import math
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


def check_terms(got, t1, t2):
    g1, g2 = got[:, 0], got[:, 1]
    e1 = np.abs(g1 - t1) / t1
    assert np.all(e1 <= 1e-5), f"T1 max rel err {float(e1.max()):.3e}"
    tol2 = 1e-5 * np.maximum(1.0, np.abs(np.log(t2))) * t2
    assert np.all(np.abs(g2 - t2) <= tol2), f"T2 max err/tol {float(np.max(np.abs(g2 - t2) / tol2)):.3e}"


def check_total(out, t1, t2):
    n = len(t1)
    ref = oracle.ise_total(t1, t2)
    scale = (np.sum(t1) + 2 * np.sum(t2)) / n
    assert abs(out[0] - ref) <= 1e-6 * scale, (out[0], ref)
    assert math.isclose(out[1], np.mean(t1), rel_tol=1e-6)
    assert math.isclose(out[2], np.mean(t2), rel_tol=1e-6)


@pytest.mark.parametrize("dx,dy,n", [(3, 1, 700), (1, 1, 257), (2, 2, 300), (5, 1, 513),
                                     (8, 2, 200), (16, 2, 140)])
def test_cv_ise_parity_all_points(dx, dy, n):
    # n = 700: 6 row blocks (ragged), 3 column blocks (ragged), 3 tiles of j
    say(f"case: cv_ise dx={dx} dy={dy} n={n}")
    v = workloads.gmm_general(n, dx + dy, seed=500 + 10 * dx + dy)
    x, y = v[:, :dx], v[:, dx:]
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    h = list(np.linspace(0.5, 0.9, dx)) + list(np.linspace(0.3, 0.45, dy))
    out, terms = m.cv_ise(h, terms=True)
    out, terms = out.cpu().numpy(), terms.cpu().numpy()
    t1, t2 = oracle.cv_ise(xo, yo, h, nthreads=NT)
    check_terms(terms, t1, t2)
    check_total(out, t1, t2)


@pytest.mark.parametrize("dx,dy", [(dx, dy) for dx in (1, 2, 3, 4, 5, 6, 7, 8, 16) for dy in (1, 2)])
def test_cv_ise_all_shapes(dx, dy):
    # every compiled (dx, dy) instance: n = 290 gives 3 row blocks and 2
    # column blocks (both ragged) and 2 tiles of j
    say(f"case: cv_ise shape dx={dx} dy={dy} n=290")
    v = workloads.gmm_general(290, dx + dy, seed=900 + 10 * dx + dy)
    x, y = v[:, :dx], v[:, dx:]
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    h = list(np.linspace(0.6, 1.0, dx)) + list(np.linspace(0.3, 0.45, dy))
    out, terms = m.cv_ise(h, terms=True)
    out, terms = out.cpu().numpy(), terms.cpu().numpy()
    t1, t2 = oracle.cv_ise(xo, yo, h, nthreads=NT)
    check_terms(terms, t1, t2)
    check_total(out, t1, t2)


def test_cv_ise_several_fold_segments_sampled():
    # n = 4,700: 19 tiles of j, three FP64 folds (8 + 8 + 3 tiles); sampled
    # points against the oracle, the total against the returned terms
    say("case: cv_ise n=4700 sampled")
    x, y = workloads.gmm(4700, seed=31, dx=2)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    h = [0.3, 0.35, 0.15]
    out, terms = m.cv_ise(h, terms=True)
    out, terms = out.cpu().numpy(), terms.cpu().numpy()
    idx = np.array([0, 1, 255, 256, 2047, 2048, 3333, 4607, 4608, 4699])
    t1, t2 = oracle.cv_ise(xo, yo, h, idx=idx, nthreads=NT)
    check_terms(terms[idx], t1, t2)
    assert math.isclose(out[1], terms[:, 0].mean(), rel_tol=1e-12)
    assert math.isclose(out[2], terms[:, 1].mean(), rel_tol=1e-12)
    assert math.isclose(out[0], out[1] - 2 * out[2], rel_tol=1e-12, abs_tol=1e-15)


def test_cv_ise_two_and_three_points():
    # n = 2: T1 = 1 / (2 sqrt(pi) hy) for both points whatever hx
    say("case: cv_ise n=2,3")
    x = np.array([[0.3], [2.0]], dtype=np.float32)
    y = np.array([[1.0], [-0.5]], dtype=np.float32)
    m = cde().Model(P.to_dev(x), P.to_dev(y))
    out, terms = m.cv_ise([0.2, 0.7], terms=True)
    terms = terms.cpu().numpy()
    assert np.allclose(terms[:, 0], 1.0 / (2.0 * math.sqrt(math.pi) * 0.7), rtol=1e-6)
    x3 = np.array([[0.0], [0.0], [0.0]], dtype=np.float32)  # identical x: uniform weights
    y3 = np.array([[0.0], [1.0], [3.0]], dtype=np.float32)
    m3 = cde().Model(P.to_dev(x3), P.to_dev(y3))
    _, terms3 = m3.cv_ise([0.5, 0.8], terms=True)
    t1, t2 = oracle.cv_ise(x3.astype(np.float64), y3.astype(np.float64), [0.5, 0.8])
    check_terms(terms3.cpu().numpy(), t1, t2)


def test_cv_ise_far_outlier_and_duplicates():
    # an x far from all others (large shift m_i) and exact duplicate rows
    say("case: cv_ise outlier and duplicates")
    rng = np.random.default_rng(3)
    x = rng.normal(size=(400, 2))
    y = rng.normal(size=(400, 1))
    x[17] = [40.0, -35.0]
    x[100:110] = x[99]
    y[100:110] = y[99]
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    h = [0.4, 0.4, 0.3]
    out, terms = m.cv_ise(h, terms=True)
    t1, t2 = oracle.cv_ise(xo, yo, h, nthreads=NT)
    check_terms(terms.cpu().numpy(), t1, t2)
    check_total(out.cpu().numpy(), t1, t2)


def test_cv_ise_rejects_bad_arguments():
    say("case: cv_ise argument checks")
    from paper_1206_5278_amd import _binding as B
    x, y = workloads.gmm(300, seed=2, dx=1)
    m64 = cde().Model(P.to_dev(x, torch.float64), P.to_dev(y, torch.float64))
    with pytest.raises(B.CdeError) as e:
        m64.cv_ise([0.5, 0.5])
    assert e.value.status == B.CDE_EUNSUPPORTED
    m32 = cde().Model(P.to_dev(x), P.to_dev(y))
    with pytest.raises(B.CdeError) as e:
        m32.cv_ise([0.5, -1.0])
    assert e.value.status == B.CDE_EINVAL
    # a later valid call still works
    out = m32.cv_ise([0.5, 0.5]).cpu().numpy()
    assert np.all(np.isfinite(out))
