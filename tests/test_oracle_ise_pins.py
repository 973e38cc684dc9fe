"""Pins of the oracle's cross-validated ISE (Section 3, eq. 2 and its
cross-validated estimate): the closed-form convolution of two y-kernels is
checked against numerical quadrature of the squared LOO density, and the
terms against closed forms, invariances and the independently pinned LOO
log-likelihood."""
import math

import numpy as np
from scipy.stats import norm

import oracle
from tests import brute


def quad_t1(x, y, hx, hy, i, pts_per_dim):
    """Integral of f^{-i}(y|x_i)^2 over y by the trapezoid rule on a grid
    reaching 10 bandwidths past the data (dy = 1 or 2)."""
    dy = y.shape[1]
    axes = [np.linspace(y[:, d].min() - 10 * hy[d], y[:, d].max() + 10 * hy[d], pts_per_dim)
            for d in range(dy)]
    if dy == 1:
        f = brute.loo_density_curve(x, y, hx, hy, i, axes[0][:, None])
        return np.trapezoid(f * f, axes[0])
    g0, g1 = np.meshgrid(axes[0], axes[1], indexing="ij")
    pts = np.stack([g0.ravel(), g1.ravel()], axis=1)
    f = brute.loo_density_curve(x, y, hx, hy, i, pts).reshape(g0.shape)
    return np.trapezoid(np.trapezoid(f * f, axes[1], axis=1), axes[0])


def test_t1_is_integral_of_squared_loo_density_dy1():
    rng = np.random.default_rng(1)
    x, y = rng.normal(size=(9, 2)), rng.normal(size=(9, 1)) * 2.0
    hx, hy = np.array([0.7, 1.1]), np.array([0.45])
    t1, t2 = oracle.cv_ise(x, y, np.concatenate([hx, hy]))
    for i in range(9):
        assert math.isclose(t1[i], quad_t1(x, y, hx, hy, i, 40001), rel_tol=1e-9), i
        f_at = brute.loo_density_curve(x, y, hx, hy, i, y[i:i + 1])[0]
        assert math.isclose(t2[i], f_at, rel_tol=1e-12), i


def test_t1_is_integral_of_squared_loo_density_dy2():
    rng = np.random.default_rng(2)
    x, y = rng.normal(size=(6, 1)), rng.normal(size=(6, 2))
    hx, hy = np.array([0.5]), np.array([0.6, 0.4])
    t1, t2 = oracle.cv_ise(x, y, np.concatenate([hx, hy]))
    for i in range(6):
        assert math.isclose(t1[i], quad_t1(x, y, hx, hy, i, 601), rel_tol=1e-8), i
        f_at = brute.loo_density_curve(x, y, hx, hy, i, y[i:i + 1])[0]
        assert math.isclose(t2[i], f_at, rel_tol=1e-12), i


def test_two_points_closed_form():
    # n = 2: f^{-i}(y|x_i) is the single y-kernel of the other point, whose
    # square integrates to 1 / (2 sqrt(pi) hy) whatever the x-bandwidth.
    x, y = np.array([[0.3], [2.0]]), np.array([[1.0], [-0.5]])
    for h in ([0.2, 0.7], [5.0, 0.05]):
        t1, t2 = oracle.cv_ise(x, y, h)
        assert np.allclose(t1, 1.0 / (2.0 * math.sqrt(math.pi) * h[1]), rtol=1e-14)
        assert np.allclose(t2, norm.pdf(1.5, scale=h[1]), rtol=1e-13)


def test_identical_x_gives_uniform_weights():
    # all x equal: every j != i has the same weight, so T1_i is the mean over
    # (j, l) != i of the sqrt(2) hy normal density of y_j - y_l
    rng = np.random.default_rng(3)
    n = 12
    x = np.full((n, 3), 0.25)
    y = rng.normal(size=(n, 1))
    hy = 0.35
    t1, t2 = oracle.cv_ise(x, y, [0.8, 0.8, 0.8, hy])
    for i in range(n):
        others = np.delete(y[:, 0], i)
        d = others[:, None] - others[None, :]
        ref = norm.pdf(d, scale=math.sqrt(2.0) * hy).sum() / (n - 1) ** 2
        assert math.isclose(t1[i], ref, rel_tol=1e-12), i
        assert math.isclose(t2[i], norm.pdf(y[i, 0] - others, scale=hy).mean(), rel_tol=1e-12)


def test_t2_is_exp_of_loo_loglik():
    rng = np.random.default_rng(4)
    x, y = rng.normal(size=(40, 3)), rng.normal(size=(40, 2))
    h = [0.6, 0.5, 0.9, 0.4, 0.3]
    _, t2 = oracle.cv_ise(x, y, h, nthreads=2)
    ell = oracle.loo(x, y, h, "cond")
    assert np.allclose(t2, np.exp(ell), rtol=1e-12)


def test_translation_and_scale():
    # moving the data changes nothing; scaling y and hy by b divides both
    # terms (densities in y) by b^dy; scaling x and hx together changes nothing
    rng = np.random.default_rng(5)
    x, y = rng.normal(size=(30, 2)), rng.normal(size=(30, 1))
    h = np.array([0.5, 0.8, 0.3])
    t1, t2 = oracle.cv_ise(x, y, h)
    s1, s2 = oracle.cv_ise(x + 7.0, y - 3.0, h)
    assert np.allclose(s1, t1, rtol=1e-9) and np.allclose(s2, t2, rtol=1e-9)
    b, a = 4.0, 0.25
    u1, u2 = oracle.cv_ise(a * x, b * y, np.concatenate([a * h[:2], b * h[2:]]))
    assert np.allclose(u1, t1 / b, rtol=1e-12) and np.allclose(u2, t2 / b, rtol=1e-12)


def test_subset_and_threads_agree():
    rng = np.random.default_rng(6)
    x, y = rng.normal(size=(80, 2)), rng.normal(size=(80, 1))
    h = [0.4, 0.4, 0.25]
    t1, t2 = oracle.cv_ise(x, y, h, nthreads=1)
    idx = np.array([0, 17, 79])
    s1, s2 = oracle.cv_ise(x, y, h, idx=idx, nthreads=3)
    assert np.array_equal(s1, t1[idx]) and np.array_equal(s2, t2[idx])
    v1, v2 = oracle.cv_ise(x, y, h, nthreads=4)
    assert np.array_equal(v1, t1) and np.array_equal(v2, t2)
    assert math.isclose(oracle.ise_total(t1, t2), t1.mean() - 2 * t2.mean(), rel_tol=1e-12)
