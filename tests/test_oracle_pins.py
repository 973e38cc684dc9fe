"""Pins of the FP64 CPU oracle against facts fixed by the paper's definitions
and by mathematics -- not against the oracle itself.

* 50-digit decimal brute force (tests/brute.py) on N <= 12, including
  bandwidths small enough that plain FP64 kernel values underflow.
* Closed forms at N = 2 and N = 3.
* Limits: hx -> inf gives the leave-one-out marginal KDE of y (a textbook
  estimator, evaluated here with scipy's normal pdf); hy -> inf gives log c_y;
  hx -> 0 gives the y-kernel at the x-nearest neighbour.
* Invariances: permutation, translation, scaling.
* JOINT - CONDITIONAL = log(c_x den_i / (n-1)), independent of hy.
* Gradient: central finite differences of the 50-digit brute force, and the
  N = 2 closed form (maximum at hy = |dy|).
* Density queries: integral over y equals 1 (Simpson), nonnegativity, the
  hx -> inf marginal KDE, and the decimal brute force.
* Thread count does not change any bit.
"""
import math

import numpy as np
import pytest
from scipy.stats import norm

import oracle
import workloads
from tests import brute

LOG2PI_2 = 0.5 * math.log(2 * math.pi)


def rand_problem(rng, n, dx, dy, scale=1.0):
    x = rng.normal(0, scale, size=(n, dx))
    y = rng.normal(0, scale, size=(n, dy))
    return x, y


@pytest.mark.parametrize("seed", range(6))
def test_decimal_bruteforce_cond_and_joint(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 13))
    dx = int(rng.integers(1, 4))
    dy = int(rng.integers(1, 3))
    x, y = rand_problem(rng, n, dx, dy)
    hx = rng.uniform(0.2, 2.0, size=dx)
    hy = rng.uniform(0.2, 2.0, size=dy)
    h = np.concatenate([hx, hy])
    for crit in ("cond", "joint"):
        got = oracle.loo(x, y, h, crit)
        ref = np.array([float(v) for v in brute.ell(x, y, hx, hy, crit)])
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)
        assert abs(oracle.total(got) - float(sum(brute.ell(x, y, hx, hy, crit)))) < 1e-12 * n


def test_decimal_bruteforce_tiny_bandwidth_underflow():
    # Kernel values near exp(-2000): a direct FP64 sum would be 0/0.  The
    # oracle's shifted form must still equal the exact 50-digit value.
    rng = np.random.default_rng(7)
    n, dx, dy = 8, 2, 1
    x, y = rand_problem(rng, n, dx, dy, scale=3.0)
    hx = np.array([0.03, 0.05])
    hy = np.array([0.04])
    got = oracle.loo(x, y, np.concatenate([hx, hy]), "cond")
    ref = np.array([float(v) for v in brute.ell(x, y, hx, hy, "cond")])
    assert np.all(np.isfinite(got))
    assert np.min(ref) < -100.0  # the regime is really extreme
    np.testing.assert_allclose(got, ref, rtol=1e-12)


def test_closed_form_n2():
    rng = np.random.default_rng(3)
    x, y = rand_problem(rng, 2, 3, 1)
    for hx in (0.1, 1.0, 7.0):
        hy = 0.6
        got = oracle.loo(x, y, [hx, hx, hx, hy], "cond")
        dyv = y[0, 0] - y[1, 0]
        expect = -math.log(hy) - LOG2PI_2 - dyv * dyv / (2 * hy * hy)
        np.testing.assert_allclose(got, [expect, expect], rtol=1e-12)
        # JOINT adds log K_hx(x1-x2) (n-1 = 1).
        gj = oracle.loo(x, y, [hx, hx, hx, hy], "joint")
        d2 = float(np.sum((x[0] - x[1]) ** 2))
        ex = expect - 3 * (math.log(hx) + LOG2PI_2) - d2 / (2 * hx * hx)
        np.testing.assert_allclose(gj, [ex, ex], rtol=1e-12)


def test_closed_form_n3():
    x = np.array([[0.0], [0.7], [-1.1]])
    y = np.array([[0.3], [-0.2], [1.4]])
    hx, hy = 0.9, 0.5

    def w(a, b):
        return math.exp(-((x[a, 0] - x[b, 0]) / hx) ** 2 / 2)

    def k(a, b):
        t = (y[a, 0] - y[b, 0]) / hy
        return math.exp(-t * t / 2) / (hy * math.sqrt(2 * math.pi))

    expect = []
    for i in range(3):
        j1, j2 = [j for j in range(3) if j != i]
        expect.append(math.log((w(i, j1) * k(i, j1) + w(i, j2) * k(i, j2)) / (w(i, j1) + w(i, j2))))
    np.testing.assert_allclose(oracle.loo(x, y, [hx, hy]), expect, rtol=1e-14)


def test_limit_hx_infinite_is_loo_marginal_kde():
    rng = np.random.default_rng(11)
    x, y = rand_problem(rng, 40, 2, 1)
    hy = 0.35
    got = oracle.loo(x, y, [1e8, 1e8, hy], "cond")
    yy = y[:, 0]
    ref = []
    for i in range(len(yy)):
        others = np.delete(yy, i)
        ref.append(math.log(np.mean(norm.pdf(yy[i], loc=others, scale=hy))))
    np.testing.assert_allclose(got, ref, rtol=1e-12)


def test_limit_hy_infinite_is_log_cy():
    rng = np.random.default_rng(12)
    x, y = rand_problem(rng, 30, 2, 2)
    got = oracle.loo(x, y, [0.5, 0.7, 1e8, 1e8], "cond")
    np.testing.assert_allclose(got, 2 * (-math.log(1e8) - LOG2PI_2), rtol=1e-14)


def test_limit_hx_zero_is_nearest_neighbour():
    rng = np.random.default_rng(13)
    gaps = rng.uniform(0.1, 0.3, size=29)
    x = np.concatenate([[0.0], np.cumsum(gaps)])
    perm = rng.permutation(30)
    x = x[perm].reshape(-1, 1)
    y = rng.normal(0, 1, size=(30, 1))
    hx, hy = 1e-3, 0.4
    got = oracle.loo(x, y, [hx, hy], "cond")
    for i in range(30):
        d = np.abs(x[:, 0] - x[i, 0])
        d[i] = np.inf
        nn = int(np.argmin(d))
        expect = norm.logpdf(y[i, 0], loc=y[nn, 0], scale=hy)
        # the shifted exponents are ~(0.1/1e-3)^2/2 = 5e3, so rounding is ~1e-12
        assert abs(got[i] - expect) < 1e-10 * max(1.0, abs(expect))


def test_invariances():
    rng = np.random.default_rng(14)
    x, y = rand_problem(rng, 60, 3, 2)
    h = np.array([0.4, 0.6, 0.5, 0.3, 0.45])
    base = oracle.loo(x, y, h, "cond")
    base_j = oracle.loo(x, y, h, "joint")
    # permutation
    p = rng.permutation(60)
    np.testing.assert_allclose(oracle.loo(x[p], y[p], h), base[p], rtol=1e-12, atol=1e-12)
    assert abs(oracle.total(oracle.loo(x[p], y[p], h)) - oracle.total(base)) < 1e-10
    # translation (by exactly representable offsets so the inputs stay exact)
    np.testing.assert_allclose(oracle.loo(x + 3.0, y - 2.0, h), base, rtol=1e-12, atol=1e-12)
    # scaling x and hx by s leaves CONDITIONAL unchanged, shifts JOINT by -dx log s
    s = 2.0
    hs = h.copy()
    hs[:3] *= s
    np.testing.assert_allclose(oracle.loo(x * s, y, hs), base, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.loo(x * s, y, hs, "joint"), base_j - 3 * math.log(s),
                               rtol=1e-12, atol=1e-12)
    # scaling y and hy by s shifts each point by -dy log s
    hs = h.copy()
    hs[3:] *= s
    np.testing.assert_allclose(oracle.loo(x, y * s, hs), base - 2 * math.log(s), rtol=1e-12,
                               atol=1e-12)


def test_joint_minus_conditional_independent_of_hy():
    rng = np.random.default_rng(15)
    x, y = rand_problem(rng, 50, 2, 1)
    diffs = []
    for hy in (0.05, 0.3, 2.0):
        h = [0.5, 0.8, hy]
        diffs.append(oracle.loo(x, y, h, "joint") - oracle.loo(x, y, h, "cond"))
    np.testing.assert_allclose(diffs[0], diffs[1], rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(diffs[0], diffs[2], rtol=1e-11, atol=1e-11)
    # and equals log(c_x den_i / (n-1)) computed directly
    hx = np.array([0.5, 0.8])
    den = np.array([sum(np.prod(norm.pdf(x[i] - x[j], scale=hx)) for j in range(50) if j != i)
                    for i in range(50)])
    np.testing.assert_allclose(diffs[0], np.log(den / 49), rtol=1e-11, atol=1e-11)


def _brute_total(x, y, h, dx, crit):
    return sum(brute.ell(x, y, h[:dx], h[dx:], crit))


@pytest.mark.parametrize("crit", ["cond", "joint"])
def test_gradient_vs_decimal_finite_differences(crit):
    rng = np.random.default_rng(16)
    n, dx, dy = 7, 2, 1
    x, y = rand_problem(rng, n, dx, dy)
    h = np.array([0.6, 0.9, 0.5])
    _, dell = oracle.loo(x, y, h, crit, grad=True)
    g = dell.sum(axis=0)
    from decimal import Decimal
    for k in range(dx + dy):
        step = Decimal("1e-12") * brute._d(h[k])
        hp = [brute._d(v) for v in h]
        hm = list(hp)
        hp[k] += step
        hm[k] -= step
        fd = (_brute_total(x, y, [float(v) for v in hp], dx, crit) -
              _brute_total(x, y, [float(v) for v in hm], dx, crit))
        # brute._d(float(...)) rounds the perturbed bandwidth; use the realised step
        realised = brute._d(float(hp[k])) - brute._d(float(hm[k]))
        fd = float(fd / realised)
        assert abs(g[k] - fd) <= 1e-7 * max(abs(fd), 1.0), (k, g[k], fd)


def test_gradient_closed_form_n2():
    x = np.array([[0.2, -0.4], [1.0, 0.3]])
    y = np.array([[0.5], [-0.3]])
    for hy in (0.3, 0.8, 1.7):
        _, dell = oracle.loo(x, y, [0.7, 0.4, hy], "cond", grad=True)
        dyv = 0.8
        np.testing.assert_allclose(dell[:, :2], 0.0, atol=1e-15)
        np.testing.assert_allclose(dell[:, 2], dyv ** 2 / hy ** 3 - 1 / hy, rtol=1e-13)
    # gradient vanishes at the maximiser hy = |dy|
    _, dell = oracle.loo(x, y, [0.7, 0.4, 0.8], "cond", grad=True)
    assert np.max(np.abs(dell[:, 2])) < 1e-14


def test_gradient_vs_fp64_finite_differences_medium():
    # Central differences with step 1e-4 relative on the FP64 oracle (the
    # finite-difference protocol used for the gradient workload).
    rng = np.random.default_rng(17)
    x, y = workloads.photoz(400, seed=3)
    h = np.array([0.05, 0.04, 0.06, 0.05, 0.07, 0.03])
    _, dell = oracle.loo(x, y, h, grad=True)
    g = dell.sum(axis=0)
    for k in range(6):
        d = 1e-4 * h[k]
        hp, hm = h.copy(), h.copy()
        hp[k] += d
        hm[k] -= d
        fd = (oracle.total(oracle.loo(x, y, hp)) - oracle.total(oracle.loo(x, y, hm))) / (2 * d)
        assert abs(g[k] - fd) <= 2e-6 * np.max(np.abs(g)), (k, g[k], fd)


def test_density_integrates_to_one_and_is_nonnegative():
    rng = np.random.default_rng(18)
    x, y = rand_problem(rng, 200, 2, 1)
    hy = 0.25
    h = [0.4, 0.5, hy]
    xq = rng.normal(0, 1, size=(5, 2))
    yg = np.linspace(y.min() - 12 * hy, y.max() + 12 * hy, 8001)  # spacing << hy
    f = oracle.density(x, y, h, xq, yg)
    assert np.all(f >= 0)
    dy = yg[1] - yg[0]
    w = np.ones_like(yg)
    w[1:-1:2] = 4
    w[2:-1:2] = 2
    integ = (f * w).sum(axis=1) * dy / 3
    np.testing.assert_allclose(integ, 1.0, atol=1e-8)


def test_density_limit_hx_infinite_and_bruteforce():
    rng = np.random.default_rng(19)
    x, y = rand_problem(rng, 25, 2, 1)
    xq = rng.normal(0, 1, size=(3, 2))
    yg = np.linspace(-2, 2, 7)
    f = oracle.density(x, y, [1e8, 1e8, 0.3], xq, yg)
    ref = np.array([[np.mean(norm.pdf(v, loc=y[:, 0], scale=0.3)) for v in yg] for _ in range(3)])
    np.testing.assert_allclose(f, ref, rtol=1e-12)
    f = oracle.density(x, y, [0.4, 0.7, 0.3], xq, yg)
    for a in range(3):
        for b in (0, 3, 6):
            ref = float(brute.density(x, y, [0.4, 0.7], [0.3], xq[a], [yg[b]]))
            assert abs(f[a, b] - ref) <= 1e-13 * max(ref, 1e-300)


def test_grid_matches_bruteforce_and_layout():
    rng = np.random.default_rng(20)
    x, y = rand_problem(rng, 9, 1, 1)
    hx = [0.3, 1.1]
    hy = [0.2, 0.5, 1.3]
    g = oracle.loo_grid(x, y, hx, hy)
    assert g.shape == (6, 9)
    for a in range(2):
        for b in range(3):
            ref = [float(v) for v in brute.ell(x, y, [hx[a]], [hy[b]])]
            np.testing.assert_allclose(g[a * 3 + b], ref, rtol=1e-13)


def test_threads_bitwise_identical_and_index_subset():
    x, y = workloads.gmm(600, seed=4)
    h = [0.3] * 5 + [0.2]
    a = oracle.loo(x, y, h, nthreads=1)
    b = oracle.loo(x, y, h, nthreads=5)
    assert np.array_equal(a, b)
    idx = [5, 0, 599, 17]
    np.testing.assert_array_equal(oracle.loo(x, y, h, idx=idx), a[idx])


def test_invalid_arguments_rejected():
    x = np.zeros((1, 1))
    with pytest.raises(ValueError):
        oracle.loo(x, x, [1.0, 1.0])
    x = np.zeros((3, 1))
    with pytest.raises(ValueError):
        oracle.loo(x, x, [0.0, 1.0])
    with pytest.raises(ValueError):
        oracle.loo(x, x, [1.0, float("nan")])
