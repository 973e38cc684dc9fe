"""Pins of the oracle's query-side products (Section 1: expectation, modes,
prediction intervals; Section 4.2: prediction by the expectation of f(y|x)
and narrowest prediction intervals of the desired coverage): the conditional
mean against a 50-digit brute force and its limits, and the density summary
against closed forms of densities whose mode and narrowest interval are
known."""
import math

import numpy as np
import pytest
from scipy.stats import norm

import oracle
from tests import brute


def test_cond_mean_decimal_bruteforce():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(9, 3))
    y = rng.normal(size=(9, 1))
    hx = [0.7, 1.1, 0.9]
    xq = rng.normal(size=(4, 3))
    got = oracle.cond_mean(x, y, hx + [0.5], xq)[:, 0]
    ref = [brute.cond_mean(x, y, hx, q) for q in xq]
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-14)


def test_cond_mean_limits_and_dy2():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(50, 2))
    y = rng.normal(size=(50, 2))
    # wide x kernel: the plain average of y; tiny x kernel: y of the x-nearest point
    wide = oracle.cond_mean(x, y, [1e8, 1e8, 1.0, 1.0], x[:3] + 0.01)
    np.testing.assert_allclose(wide, np.tile(y.mean(0), (3, 1)), rtol=1e-12)
    q = x[:3] + 1e-4
    tiny = oracle.cond_mean(x, y, [1e-3, 1e-3, 1.0, 1.0], q)
    nn = [np.argmin(((x - qq) ** 2).sum(1)) for qq in q]
    np.testing.assert_allclose(tiny, y[nn], rtol=1e-12)
    # constant y: the mean is that constant whatever the weights
    c = oracle.cond_mean(x, np.full((50, 1), 2.5), [0.3, 0.3, 1.0], rng.normal(size=(5, 2)))
    np.testing.assert_allclose(c, 2.5, rtol=1e-14)


def test_summary_gaussian_closed_form():
    # N(mu, s) on a fine grid: mass ~ 1, mode mu, narrowest 95% interval mu +- 1.96 s
    mu, s = 1.0, 1.5
    yg = np.linspace(-8, 10, 9001)
    step = yg[1] - yg[0]
    out = oracle.density_summary(norm.pdf(yg, mu, s)[None], yg, 0.05)[0]
    assert abs(out[0] - (norm.cdf(10, mu, s) - norm.cdf(-8, mu, s))) < 1e-6
    assert abs(out[1] - mu) <= step / 2
    z = norm.ppf(0.975)
    assert abs(out[2] - (mu - z * s)) < 2 * step and abs(out[3] - (mu + z * s)) < 2 * step


def test_summary_uniform_ties_and_bimodal():
    # uniform on [0, 1] (grid ending at 1): every interval of length 0.9 is
    # narrowest; the first candidate in order starts at the grid's first point
    yg = np.linspace(0.0, 1.0, 1001)
    out = oracle.density_summary(np.ones((1, 1001)), yg, 0.1)[0]
    assert abs(out[0] - 1.0) < 1e-12 and out[1] == 0.0
    assert out[2] == 0.0 and abs(out[3] - 0.9) < 1e-12
    # 0.7 N(-3, 0.5) + 0.3 N(3, 0.5): the narrowest 50% interval is inside the heavier mode
    yg = np.linspace(-8, 8, 16001)
    f = 0.7 * norm.pdf(yg, -3, 0.5) + 0.3 * norm.pdf(yg, 3, 0.5)
    out = oracle.density_summary(f[None], yg, 0.5)[0]
    assert abs(out[1] + 3) < 1e-3
    # half-width w with 0.7 (2 Phi(w/0.5) - 1) = 0.5
    w = 0.5 * norm.ppf((0.5 / 0.7 + 1) / 2)
    assert abs(out[2] - (-3 - w)) < 2e-3 and abs(out[3] - (-3 + w)) < 2e-3


def test_summary_linear_density_exact():
    # f(y) = y on [0, 1]: the trapezoid rule is exact (mass 1/2), the mode is
    # the last grid point, and G(y) = y^2 at the nodes; the narrowest 80%
    # interval of the increasing density ends at 1 and starts at sqrt(0.2)
    # (interpolated between the nodes 0.4 and 0.5)
    yl = np.linspace(0.0, 1.0, 11)
    out = oracle.density_summary(yl[None], yl, 0.2)[0]
    assert abs(out[0] - 0.5) < 1e-15 and out[1] == 1.0 and out[3] == 1.0
    lo_nodes = 0.4 + (0.2 - 0.16) / (0.25 - 0.16) * 0.1
    assert abs(out[2] - lo_nodes) < 1e-12


def test_summary_zero_mass_row():
    yg = np.linspace(0, 1, 5)
    out = oracle.density_summary(np.zeros((1, 5)), yg, 0.05)[0]
    assert out[0] == 0.0 and out[1] == 0.0 and math.isnan(out[2]) and math.isnan(out[3])


def test_summary_of_oracle_density_brackets_the_mean():
    # the density of eq. (1) from the oracle, summarised: the interval holds
    # the conditional mean for a unimodal case, and the mass is ~1
    rng = np.random.default_rng(4)
    x = rng.normal(size=(200, 1))
    y = 0.5 * x + 0.1 * rng.normal(size=(200, 1))
    h = [0.3, 0.2]
    xq = np.array([[0.2]])
    yg = np.linspace(y.min() - 2, y.max() + 2, 4001)
    out = oracle.density_summary(oracle.density(x, y, h, xq, yg), yg, 0.05)[0]
    m = oracle.cond_mean(x, y, h, xq)[0, 0]
    assert abs(out[0] - 1.0) < 1e-6 and out[2] < m < out[3]
