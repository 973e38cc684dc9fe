"""GPU parity of the query-side products against the FP64 oracle, through the
C ABI: the conditional mean (both precisions, several shapes, multi-chunk
training sets, wide and tiny bandwidths) and the density summary (bit-equal
to the oracle's scalar definition, on oracle-made and GPU-made densities)."""
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


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("dx,dy", [(1, 1), (2, 2), (5, 1), (16, 2)])
def test_conditional_mean_parity(dx, dy, dtype):
    say(f"case: conditional mean dx={dx} dy={dy} {dtype}")
    v = workloads.gmm_general(3000, dx + dy, seed=400 + dx + dy)
    x, y = v[:, :dx], v[:, dx:]
    if dtype == torch.float32:
        xo, yo, xd, yd = P.f32_pair(x, y)
    else:
        xo, yo = x, y
        xd, yd = P.to_dev(xo, torch.float64), P.to_dev(yo, torch.float64)
    m = cde().Model(xd, yd)
    rng = np.random.default_rng(dx)
    xq = xo[rng.choice(3000, 333)] + 0.1 * rng.normal(size=(333, dx))
    xq = xq.astype(np.float32).astype(np.float64) if dtype == torch.float32 else xq
    for hs in (0.5, 3.0, 0.02):
        h = [hs] * dx + [0.4] * dy
        got = m.conditional_mean(P.to_dev(xq, dtype), h).cpu().numpy()
        ref = oracle.cond_mean(xo, yo, h, xq)
        scale = np.abs(yo).max()
        assert np.all(np.abs(got - ref) <= 1e-12 * scale), float(np.max(np.abs(got - ref)))


@pytest.mark.parametrize("n", [1001, 1026])
def test_query_and_mean_ragged_tail(n):
    # The shift prepasses screen four training rows per branch and the rows
    # of a tile beyond a multiple of four one at a time.  Here the last tile
    # holds n % 256 rows (233 and 2), and some queries sit on the last
    # training point, so their nearest neighbour, which fixes the shift, is
    # one of those single rows; a tiny bandwidth makes a wrong shift visible.
    say(f"case: query and conditional mean, ragged tail n={n}")
    x, y = workloads.gmm(n, seed=21, dx=3)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    rng = np.random.default_rng(n)
    xq = np.concatenate([xo[n - 1:n], xo[n - 1:n] + 1e-3, xo[rng.choice(n, 13)] + 0.05 * rng.normal(size=(13, 3))])
    xq = xq.astype(np.float32).astype(np.float64)
    yg = np.linspace(yo.min() - 1, yo.max() + 1, 70).astype(np.float32).astype(np.float64)
    for hs in (0.4, 0.01):
        h = [hs] * 3 + [0.3]
        f = m.query(P.to_dev(xq), P.to_dev(yg), h).cpu().numpy()
        ref = oracle.density(xo, yo, h, xq, yg, nthreads=NT)
        peak = ref.max(axis=1, keepdims=True)
        err = np.abs(f - ref)
        assert np.all(err <= 1e-5 * ref + 1e-7 * peak), float(np.max(err / (1e-5 * ref + 1e-7 * peak)))
        got = m.conditional_mean(P.to_dev(xq, torch.float32), h).cpu().numpy()
        ref_m = oracle.cond_mean(xo, yo, h, xq)
        assert np.all(np.abs(got - ref_m) <= 1e-12 * np.abs(yo).max()), float(np.max(np.abs(got - ref_m)))
    m.close()


def test_conditional_mean_large_set_slices():
    # 70,000 training points (64 chunks) and 20,000 queries (two slices)
    say("case: conditional mean n=70000 q=20000")
    x, y = workloads.gmm(70_000, seed=14, dx=3)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    rng = np.random.default_rng(7)
    xq = (xo[rng.choice(70_000, 20_000)] + 0.05).astype(np.float32)
    got = m.conditional_mean(P.to_dev(xq, torch.float32), [0.3, 0.3, 0.3, 0.2]).cpu().numpy()
    idx = [0, 9_999, 16_384, 19_999]
    ref = oracle.cond_mean(xo, yo, [0.3, 0.3, 0.3, 0.2], xq[idx].astype(np.float64))
    np.testing.assert_allclose(got[idx], ref, rtol=0, atol=1e-12 * np.abs(yo).max())


def test_density_summary_bit_equal_to_oracle():
    say("case: density summary vs oracle")
    rng = np.random.default_rng(8)
    x = rng.normal(size=(400, 2))
    y = np.sin(2 * x[:, :1]) + 0.3 * rng.normal(size=(400, 1))
    h = [0.3, 0.3, 0.15]
    xq = rng.normal(size=(50, 2))
    yg = np.linspace(-3, 3, 777)
    f = oracle.density(x, y, h, xq, yg, nthreads=NT)
    f = np.vstack([f, np.zeros((1, 777)), np.ones((1, 777)), np.linspace(0, 1, 777)[None]])
    for alpha in (0.05, 0.5, 0.9):
        ref = oracle.density_summary(f, yg, alpha)
        got = cde().density_summary(P.to_dev(f, torch.float64), yg, alpha).cpu().numpy()
        assert np.array_equal(got, ref, equal_nan=True), np.nanmax(np.abs(got - ref))


@pytest.mark.parametrize("k,q", [(2, 5), (3, 9), (256, 4099), (2048, 7), (4096, 3)])
def test_density_summary_sizes(k, q):
    # grid sizes that give 4, 2 and 1 rows per block, ragged last blocks, and
    # rows with ties (flat stretches) and zero mass
    say(f"case: density summary k={k} q={q}")
    rng = np.random.default_rng(k + q)
    yg = np.sort(rng.uniform(-4.0, 4.0, k))
    yg[0], yg[-1] = -4.0, 4.0
    centres = rng.uniform(-2.0, 2.0, (q, 1))
    f = np.exp(-0.5 * ((yg[None, :] - centres) / 0.7) ** 2)
    f[::3] = np.round(f[::3], 2)  # flat stretches: ties in the mode and the widths
    if q > 1:
        f[1] = 0.0
    for alpha in (0.05, 0.3):
        ref = oracle.density_summary(f, yg, alpha)
        got = cde().density_summary(P.to_dev(f, torch.float64), yg, alpha).cpu().numpy()
        assert np.array_equal(got, ref, equal_nan=True), np.nanmax(np.abs(got - ref))


def test_density_summary_of_gpu_query_rows():
    # the GPU query feeds the GPU summary; the summary of the oracle's density
    # at the same queries agrees within the query tolerance's effect
    say("case: GPU query -> summary")
    x, y = workloads.gmm(5000, seed=15, dx=2)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    h = [0.4, 0.4, 0.3]
    rng = np.random.default_rng(2)
    xq = (xo[rng.choice(5000, 64)] + 0.1).astype(np.float32)
    yg = np.linspace(yo.min() - 2, yo.max() + 2, 512).astype(np.float32)
    f = m.query(P.to_dev(xq, torch.float32), P.to_dev(yg, torch.float32), h)
    got = cde().density_summary(f, yg.astype(np.float64), 0.05).cpu().numpy()
    ref = oracle.density_summary(oracle.density(xo, yo, h, xq.astype(np.float64), yg.astype(np.float64),
                                                nthreads=NT), yg.astype(np.float64), 0.05)
    step = float(yg[1] - yg[0])
    np.testing.assert_allclose(got[:, 0], ref[:, 0], rtol=1e-5)
    assert np.all(np.abs(got[:, 2:] - ref[:, 2:]) <= 0.05 * step + 1e-9)
    # the mode can only move between grid points of (near-)equal density
    assert np.all(np.abs(got[:, 1] - ref[:, 1]) <= 2 * step)


def test_summary_rejects_bad_arguments():
    from paper_1206_5278_amd import _binding as B
    lib = B.load()
    assert lib.cde_density_summary(None, None, 1, 1, 0.05, None, None) == B.CDE_EINVAL
    assert lib.cde_density_summary(8, 8, 1, 4, 1.5, 8, None) == B.CDE_EINVAL
    assert lib.cde_density_summary(None, None, 0, 4, 0.05, None, None) == B.CDE_OK
