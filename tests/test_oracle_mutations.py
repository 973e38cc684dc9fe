"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake (a dropped term, a wrong sign, index or stride,
a missing constant) in a temporary copy of the oracle's C source, builds it,
and checks that the compact battery of independent pins below rejects it.
Everything runs on the CPU; the committed oracle is never modified.
"""
import math
import os

import numpy as np
import pytest
from scipy.stats import norm

import oracle
from tests import brute

SRC = os.path.join(os.path.dirname(oracle.__file__), "cde_oracle.c")

MUTATIONS = {
    "self_pair_included": ("if (j == i) continue;", ""),
    "wrong_sign_y_exponent": ("ab[j] = -0.5 * sx - 0.5 * sy;", "ab[j] = -0.5 * sx + 0.5 * sy;"),
    "missing_2pi_constant": ("s -= log(h[k]) + HALF_LOG_2PI;", "s -= log(h[k]);"),
    "y_scaled_by_hx": ("double t = (yi[l] - yj[l]) / hy[l];", "double t = (yi[l] - yj[l]) / hx[l];"),
    "wrong_x_stride": ("const double* xj = J->x + (size_t)j * dx;",
                       "const double* xj = J->x + (size_t)j * dy;"),
    "grad_sign": ("grad[k] = (mv / U - mw / D) / h3;", "grad[k] = (mv / U + mw / D) / h3;"),
    "grad_missing_norm_term": ("grad[dx + l] = (mvy / U) / h3 - 1.0 / hy[l];",
                               "grad[dx + l] = (mvy / U) / h3;"),
    "joint_wrong_count": ("- log((double)(n - 1));", "- log((double)n);"),
    "density_missing_cy": ("exp(lcy + (Mxy + log(U)) - (Mx + log(D)))",
                           "exp((Mxy + log(U)) - (Mx + log(D)))"),
    "density_den_shift_dropped": ("J->f[(size_t)qq * J->k + g] = exp(lcy + (Mxy + log(U)) - (Mx + log(D)));",
                                  "J->f[(size_t)qq * J->k + g] = exp(lcy + (Mxy + log(U)) - log(D));"),
}


# Mistakes planted in the Epanechnikov kernel's code.
EPAN_MUTATIONS = {
    "epan_norm_missing_half": ("double s = log((d + 2.0) / 2.0) - log_vd;",
                               "double s = log(d + 2.0) - log_vd;"),
    "epan_ball_volume_exponent": ("0.5 * d * log(PI) - lgamma(0.5 * d + 1.0)",
                                  "d * log(PI) - lgamma(0.5 * d + 1.0)"),
    "epan_y_window_uses_x": ("        const double wy = sy < 1.0 ? 1.0 - sy : 0.0;\n        D += wx;\n        U += wx * wy;\n    }\n    const double lcy",
                             "        const double wy = sy < 1.0 ? 1.0 - sx : 0.0;\n        D += wx;\n        U += wx * wy;\n    }\n    const double lcy"),
    "epan_den_weighted_by_y": ("        D += wx;\n        U += wx * wy;\n    }\n    const double lcy",
                               "        D += wx * wy;\n        U += wx * wy;\n    }\n    const double lcy"),
    "epan_window_not_squared": ("            double t = (xi[k] - xj[k]) / hx[k];\n            sx += t * t;\n        }\n        for (int l = 0; l < dy; ++l) {\n            double t = (yi[l] - yj[l]) / hy[l];\n            sy += t * t;\n        }\n        const double wx",
                                "            double t = (xi[k] - xj[k]) / hx[k];\n            sx += fabs(t);\n        }\n        for (int l = 0; l < dy; ++l) {\n            double t = (yi[l] - yj[l]) / hy[l];\n            sy += t * t;\n        }\n        const double wx"),
    "epan_joint_missing_cx": ("*ell = log_norm_epan(hx, dx) + lcy + log(U) - log((double)(n - 1));",
                              "*ell = lcy + log(U) - log((double)(n - 1));"),
    "epan_self_pair_included": ("    double D = 0.0, U = 0.0;\n    for (long j = 0; j < n; ++j) {\n        if (j == i) continue;           /* leave point i out (eq. 3) */",
                                "    double D = 0.0, U = 0.0;\n    for (long j = 0; j < n; ++j) {\n"),
}


def battery_epan(lib) -> list:
    """Independent Epanechnikov checks; returns the names of those that fail."""
    failed = []
    rng = np.random.default_rng(8)
    n, dx, dy = 9, 2, 1
    x = rng.normal(0, 1, size=(n, dx))
    y = rng.normal(0, 1, size=(n, dy))
    hx, hy = np.array([1.8, 2.2]), np.array([1.6])
    h = np.concatenate([hx, hy])
    for crit in ("cond", "joint"):
        got = oracle.loo_epan(x, y, h, crit, lib=lib)
        ref = np.array(brute.ell_epan(x, y, hx, hy, crit))
        if not (np.array_equal(np.isfinite(got), np.isfinite(ref)) and
                np.allclose(got[np.isfinite(ref)], ref[np.isfinite(ref)], rtol=1e-12, atol=1e-12)):
            failed.append(f"epan_brute_{crit}")
    xq = rng.normal(0, 1, size=(1, dx))
    yg = np.linspace(y.min() - 2.0, y.max() + 2.0, 20001)
    f = oracle.density_epan(x, y, h, xq, yg, lib=lib)
    if abs(np.trapezoid(f[0], yg) - 1.0) > 1e-6:
        failed.append("epan_density_integral")
    return failed


# Mistakes planted in the query-side products.
PRODUCT_MUTATIONS = {
    "mean_unweighted": ("S += w * y[(size_t)i * dy + l];", "S += y[(size_t)i * dy + l];"),
    "summary_left_rule": ("c += (r[g] + r[g + 1]) * 0.5 * (yg[g + 1] - yg[g]);",
                          "c += r[g] * (yg[g + 1] - yg[g]);"),
    "summary_mode_last_max": ("if (r[g] > r[imax]) imax = g;", "if (r[g] >= r[imax]) imax = g;"),
    "summary_wrong_coverage": ("const double p = G[g] + cover;", "const double p = G[g] + alpha;"),
}


def battery_products(lib) -> list:
    """Independent checks of the conditional mean and the density summary."""
    from scipy.stats import norm as _norm
    failed = []
    rng = np.random.default_rng(12)
    x = rng.normal(size=(8, 2))
    y = rng.normal(size=(8, 1))
    xq = rng.normal(size=(2, 2))
    got = oracle.cond_mean(x, y, [0.8, 1.2, 0.5], xq, lib=lib)[:, 0]
    ref = [brute.cond_mean(x, y, [0.8, 1.2], q) for q in xq]
    if not np.allclose(got, ref, rtol=1e-12, atol=1e-13):
        failed.append("mean_brute")
    yg = np.linspace(-8, 10, 9001)
    out = oracle.density_summary(_norm.pdf(yg, 1.0, 1.5)[None], yg, 0.05, lib=lib)[0]
    z = _norm.ppf(0.975)
    if abs(out[0] - 1.0) > 1e-6 or abs(out[2] - (1 - z * 1.5)) > 0.01 or abs(out[3] - (1 + z * 1.5)) > 0.01:
        failed.append("summary_gaussian")
    yu = np.linspace(0.0, 1.0, 101)
    out = oracle.density_summary(np.ones((1, 101)), yu, 0.1, lib=lib)[0]
    if out[1] != 0.0:
        failed.append("summary_uniform_mode")
    yl = np.linspace(0.0, 1.0, 11)  # f(y) = y: the trapezoid rule is exact, mass 1/2
    out = oracle.density_summary(yl[None], yl, 0.1, lib=lib)[0]
    if abs(out[0] - 0.5) > 1e-14:
        failed.append("summary_linear_mass")
    return failed


# Mistakes planted in the cross-validated ISE.
ISE_MUTATIONS = {
    "ise_convolution_width_h": ("inner += w[l] * exp(-0.25 * s);", "inner += w[l] * exp(-0.5 * s);"),
    "ise_convolution_norm_sqrt2pi": ("cg /= 2.0 * sqrt(PI) * hy[l];", "cg /= sqrt(2.0 * PI) * hy[l];"),
    "ise_l_equal_i_kept": ("            if (l == i) continue;\n", ""),
    "ise_den_not_squared": ("*t1 = cg * Q / (W * W);", "*t1 = cg * Q / W;"),
    "ise_t2_missing_cy": ("*t2 = cy * num / W;", "*t2 = num / W;"),
    "ise_pair_uses_point_y": ("double t = (yj[d] - yl[d]) / hy[d];", "double t = (yi[d] - yl[d]) / hy[d];"),
    "ise_inner_unweighted": ("inner += w[l] * exp(-0.25 * s);", "inner += exp(-0.25 * s);"),
}


def battery_ise(lib) -> list:
    """Independent checks of the cross-validated ISE terms (quadrature of the
    squared LOO density, the LOO density at the point)."""
    failed = []
    rng = np.random.default_rng(14)
    x, y = rng.normal(size=(6, 2)), rng.normal(size=(6, 1))
    hx, hy = np.array([0.9, 0.6]), np.array([0.5])
    t1, t2 = oracle.cv_ise(x, y, np.concatenate([hx, hy]), lib=lib)
    for i in range(6):
        yy = np.linspace(y.min() - 10 * hy[0], y.max() + 10 * hy[0], 20001)
        f = brute.loo_density_curve(x, y, hx, hy, i, yy[:, None])
        if not math.isclose(t1[i], np.trapezoid(f * f, yy), rel_tol=1e-8):
            failed.append(f"t1_quadrature_{i}")
        if not math.isclose(t2[i], brute.loo_density_curve(x, y, hx, hy, i, y[i:i + 1])[0],
                            rel_tol=1e-12):
            failed.append(f"t2_point_{i}")
    return failed


def battery(lib) -> list:
    """Independent checks; returns the names of those that fail."""
    failed = []
    rng = np.random.default_rng(5)
    n, dx, dy = 7, 2, 1
    x = rng.normal(0, 2, size=(n, dx))
    y = rng.normal(0, 1, size=(n, dy))
    hx, hy = np.array([0.7, 1.2]), np.array([0.5])
    h = np.concatenate([hx, hy])
    for crit in ("cond", "joint"):
        got = oracle.loo(x, y, h, crit, lib=lib)
        ref = np.array([float(v) for v in brute.ell(x, y, hx, hy, crit)])
        if not np.allclose(got, ref, rtol=1e-12, atol=1e-12):
            failed.append(f"brute_{crit}")
    # gradient: central differences of the 50-digit brute force
    _, dell = oracle.loo(x, y, h, "cond", grad=True, lib=lib)
    g = dell.sum(axis=0)
    for k in range(3):
        hp, hm = h.copy(), h.copy()
        d = 1e-6 * h[k]
        hp[k] += d
        hm[k] -= d
        fd = (sum(float(v) for v in brute.ell(x, y, hp[:2], hp[2:])) -
              sum(float(v) for v in brute.ell(x, y, hm[:2], hm[2:]))) / (hp[k] - hm[k])
        if abs(g[k] - fd) > 1e-6 * max(1.0, abs(fd)):
            failed.append(f"grad_{k}")
            break
    # density: integral over y is 1 and matches the brute force
    xq = rng.normal(0, 1, size=(2, dx))
    yg = np.linspace(y.min() - 8 * hy[0], y.max() + 8 * hy[0], 2001)
    f = oracle.density(x, y, h, xq, yg, lib=lib)
    integ = np.trapezoid(f, yg, axis=1)
    if not np.allclose(integ, 1.0, atol=1e-6):
        failed.append("density_integral")
    ref = float(brute.density(x, y, hx, hy, xq[0], [yg[1000]]))
    if abs(f[0, 1000] - ref) > 1e-12 * ref:
        failed.append("density_brute")
    # hx -> infinity limit (LOO marginal KDE of y)
    got = oracle.loo(x, y, [1e8, 1e8, hy[0]], lib=lib)
    ref = [math.log(np.mean(norm.pdf(y[i, 0], loc=np.delete(y[:, 0], i), scale=hy[0])))
           for i in range(n)]
    if not np.allclose(got, ref, rtol=1e-12):
        failed.append("limit_hx_inf")
    return failed


def test_unmutated_oracle_passes_battery():
    assert battery(None) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert old in src, f"mutation anchor not found: {old!r}"
    mutated = tmp_path / "mut.c"
    mutated.write_text(src.replace(old, new))
    so = oracle.build(str(mutated), str(tmp_path / "libmut.so"))
    lib = oracle.load_library(so)
    assert battery(lib), f"mutation {name} was not detected by any pin"


def test_unmutated_oracle_passes_epan_battery():
    assert battery_epan(None) == []


@pytest.mark.parametrize("name", sorted(EPAN_MUTATIONS))
def test_planted_epan_mistake_is_caught(name, tmp_path):
    old, new = EPAN_MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique: {old!r}"
    mutated = tmp_path / "mut.c"
    mutated.write_text(src.replace(old, new))
    so = oracle.build(str(mutated), str(tmp_path / "libmut.so"))
    lib = oracle.load_library(so)
    assert battery_epan(lib), f"mutation {name} was not detected by any pin"


def test_unmutated_oracle_passes_products_battery():
    assert battery_products(None) == []


@pytest.mark.parametrize("name", sorted(PRODUCT_MUTATIONS))
def test_planted_product_mistake_is_caught(name, tmp_path):
    old, new = PRODUCT_MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique: {old!r}"
    mutated = tmp_path / "mut.c"
    mutated.write_text(src.replace(old, new))
    so = oracle.build(str(mutated), str(tmp_path / "libmut.so"))
    lib = oracle.load_library(so)
    assert battery_products(lib), f"mutation {name} was not detected by any pin"


def test_unmutated_oracle_passes_ise_battery():
    assert battery_ise(None) == []


@pytest.mark.parametrize("name", sorted(ISE_MUTATIONS))
def test_planted_ise_mistake_is_caught(name, tmp_path):
    old, new = ISE_MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique: {old!r}"
    mutated = tmp_path / "mut.c"
    mutated.write_text(src.replace(old, new))
    so = oracle.build(str(mutated), str(tmp_path / "libmut.so"))
    lib = oracle.load_library(so)
    assert battery_ise(lib), f"mutation {name} was not detected by any pin"
