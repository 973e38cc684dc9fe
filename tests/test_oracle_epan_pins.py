"""Pins of the oracle's Epanechnikov kernel (Section 4's kernel, radial over
bandwidth-scaled coordinates, multivariate normalisation), each against
something other than the oracle itself: a 50-digit brute force whose unit-ball
volume comes from its own recurrence, closed forms, the LOO kernel density
estimate it reduces to, the normalisation of the density, invariances, and
the divergence at tiny bandwidths noted in Section 4.1."""
import math

import numpy as np
import pytest

import oracle
from tests import brute


@pytest.mark.parametrize("dx,dy", [(1, 1), (2, 1), (3, 2)])
@pytest.mark.parametrize("crit", ["cond", "joint"])
def test_epan_decimal_bruteforce(dx, dy, crit):
    rng = np.random.default_rng(10 * dx + dy)
    n = 11
    x = rng.normal(0, 1, size=(n, dx))
    y = rng.normal(0, 1, size=(n, dy))
    hx = rng.uniform(1.5, 2.5, size=dx)
    hy = rng.uniform(1.5, 2.5, size=dy)
    got = oracle.loo_epan(x, y, np.concatenate([hx, hy]), crit)
    ref = np.array(brute.ell_epan(x, y, hx, hy, crit))
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin)
    assert np.all(got[~fin] == -np.inf)
    assert fin.sum() >= n - 2
    np.testing.assert_allclose(got[fin], ref[fin], rtol=1e-13, atol=1e-13)


def test_epan_closed_form_two_points():
    # n = 2: each point sees only the other, so l = log K_hy(dy) when the x
    # distance is inside the window, else -inf (0/0 and 0 both diverge).
    x = np.array([[0.0], [0.3]])
    y = np.array([[1.0], [1.4]])
    for hx, hy, expect in [(0.5, 0.5, math.log(0.75 / 0.5 * (1 - (0.4 / 0.5) ** 2))),
                           (0.5, 0.3, -math.inf), (0.2, 0.5, -math.inf),
                           (10.0, 2.0, math.log(0.75 / 2.0 * (1 - 0.04)))]:
        got = oracle.loo_epan(x, y, [hx, hy])
        assert got[0] == got[1]
        if math.isinf(expect):
            assert got[0] == -math.inf
        else:
            assert abs(got[0] - expect) <= 1e-14 * abs(expect) + 1e-15


def test_epan_hx_infinite_is_loo_epanechnikov_kde():
    # Every x weight tends to 1: l_i is the log of the LOO Epanechnikov kernel
    # density estimate of y_i (textbook form, coded here separately).
    rng = np.random.default_rng(3)
    n = 40
    x = rng.normal(size=(n, 2))
    y = rng.normal(size=(n, 1))
    hy = 0.9
    got = oracle.loo_epan(x, y, [1e8, 1e8, hy])
    for i in range(n):
        u = (y[i, 0] - np.delete(y[:, 0], i)) / hy
        kde = np.mean(np.where(np.abs(u) < 1, 0.75 * (1 - u * u) / hy, 0.0))
        ref = math.log(kde) if kde > 0 else -math.inf
        assert abs(got[i] - ref) <= 1e-12 * max(1.0, abs(ref)) or got[i] == ref


def test_epan_density_normalised_dy1_and_dy2():
    # f(y|x) integrates to 1 over y: pins c_1 = 3/4 and c_2 = 2/pi.
    rng = np.random.default_rng(4)
    x = rng.normal(size=(30, 2))
    y1 = rng.normal(size=(30, 1))
    yg = np.linspace(y1.min() - 1.0, y1.max() + 1.0, 20001)
    f = oracle.density_epan(x, y1, [1.2, 1.2, 0.6], x[:3] + 0.1, yg)
    assert np.all(f >= 0)
    np.testing.assert_allclose(np.trapezoid(f, yg, axis=1), 1.0, atol=2e-7)
    y2 = rng.normal(size=(30, 2))
    g1 = np.linspace(y2[:, 0].min() - 0.8, y2[:, 0].max() + 0.8, 601)
    g2 = np.linspace(y2[:, 1].min() - 0.8, y2[:, 1].max() + 0.8, 601)
    Y1, Y2 = np.meshgrid(g1, g2, indexing="ij")
    grid = np.stack([Y1.ravel(), Y2.ravel()], axis=1)
    f2 = oracle.density_epan(x, y2, [1.2, 1.2, 0.7, 0.6], x[:1] + 0.1, grid).reshape(601, 601)
    integ = np.trapezoid(np.trapezoid(f2, g2, axis=1), g1)
    assert abs(integ - 1.0) < 2e-4


def test_epan_invariances_and_divergence():
    rng = np.random.default_rng(6)
    n = 60
    x = rng.normal(size=(n, 2))
    y = rng.normal(size=(n, 1))
    h = [0.8, 0.9, 0.7]
    base = oracle.loo_epan(x, y, h)
    perm = rng.permutation(n)
    np.testing.assert_allclose(oracle.loo_epan(x[perm], y[perm], h), base[perm], rtol=1e-13)
    np.testing.assert_allclose(oracle.loo_epan(x + 3.0, y - 2.0, h), base, rtol=1e-12, atol=1e-12)
    # scaling (x, hx) by s leaves the conditional value unchanged
    np.testing.assert_allclose(oracle.loo_epan(2.5 * x, y, [2.0, 2.25, 0.7]), base, rtol=1e-12,
                               atol=1e-12)
    # scaling (y, hy) by s shifts every finite value by -log s (dy = 1)
    sc = oracle.loo_epan(x, 4.0 * y, [0.8, 0.9, 2.8])
    fin = np.isfinite(base)
    np.testing.assert_allclose(sc[fin], base[fin] - math.log(4.0), rtol=1e-12, atol=1e-12)
    # tiny bandwidths: isolated points diverge, and so does the total
    tiny = oracle.loo_epan(x, y, [1e-3, 1e-3, 1e-3])
    assert np.all(tiny == -np.inf)
    assert oracle.total(tiny) == -np.inf
    # joint - conditional = log(c_x D / (n-1)) does not depend on hy
    with np.errstate(invalid="ignore"):
        j1 = oracle.loo_epan(x, y, h, "joint") - oracle.loo_epan(x, y, h, "cond")
        j2 = (oracle.loo_epan(x, y, [0.8, 0.9, 1.9], "joint")
              - oracle.loo_epan(x, y, [0.8, 0.9, 1.9], "cond"))
    both = np.isfinite(j1) & np.isfinite(j2)
    np.testing.assert_allclose(j1[both], j2[both], rtol=1e-12, atol=1e-12)
