"""GPU parity of the scalar-bandwidth grid path (MFMA kernel on FP32 models)
against the FP64 oracle evaluated setting by setting, through the C ABI."""
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


def run_grid(x, y, hx, hy, crit="cond"):
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    tot, pp, nonfin = m.loo_grid(hx, hy, crit, per_point=True)
    ref = oracle.loo_grid(xo, yo, hx, hy, crit, nthreads=NT)
    return m, tot.cpu().numpy(), pp.cpu().numpy(), int(nonfin.item()), ref


def check(tot, pp, ref):
    P.assert_points(pp, ref)
    for s in range(ref.shape[0]):
        P.assert_total(float(tot[s]), oracle.total(ref[s]), ref[s])


SHAPES = [(dx, dy) for dx in (1, 2, 3, 4, 5, 6, 7, 8, 16) for dy in (1, 2)]


@pytest.mark.parametrize("dx,dy", SHAPES)
def test_grid_all_shapes_padded_grid(dx, dy):
    print(f"case: grid shape dx={dx} dy={dy} n=300 grid 5x7", flush=True)
    v = workloads.gmm_general(300, dx + dy, seed=100 + dx * 10 + dy)
    hx = workloads.geomspace(0.2, 3.0, 5)
    hy = workloads.geomspace(0.1, 2.0, 7)
    _, tot, pp, nonfin, ref = run_grid(v[:, :dx], v[:, dx:], hx, hy)
    assert nonfin == 0
    check(tot, pp, ref)


@pytest.mark.parametrize("crit", ["cond", "joint"])
def test_grid_ragged_16x16(crit):
    print(f"case: grid ragged n=700 16x16 {crit}", flush=True)
    x, y = workloads.gmm(700, seed=21)
    hx = hy = workloads.geomspace(0.05, 5.0, 16)
    _, tot, pp, nonfin, ref = run_grid(x, y, hx, hy, crit)
    assert nonfin == 0
    check(tot, pp, ref)


def test_grid_32x32_small_n():
    print("case: grid n=1100 32x32", flush=True)
    x, y = workloads.gmm(1100, seed=22)
    hx = hy = workloads.geomspace(0.05, 5.0, 32)
    _, tot, pp, nonfin, ref = run_grid(x, y, hx, hy)
    assert nonfin == 0
    check(tot, pp, ref)


@pytest.mark.parametrize("gx,gy,descending", [(17, 64, False), (64, 20, True), (33, 40, False)])
def test_grid_quad_tiles_ragged_and_bias_placement(gx, gy, descending):
    # grids whose padded sides are multiples of 32 run on 2 x 2 tile quads
    # (17 x 64, 64 x 20); 33 x 40 pads to 48 x 48 and runs one tile per
    # block.  A descending hx list puts the smallest hx (the biased a-tile)
    # in the last tile of its quad.
    print(f"case: grid quads n=800 {gx}x{gy} descending={descending}", flush=True)
    x, y = workloads.gmm(800, seed=23, dx=2)
    hx = workloads.geomspace(0.03, 4.0, gx)
    hy = workloads.geomspace(0.03, 3.0, gy)
    if descending:
        hx = hx[::-1].copy()
    _, tot, pp, nonfin, ref = run_grid(x, y, hx, hy)
    assert nonfin == 0
    check(tot, pp, ref)


@pytest.mark.parametrize("dx,dy", [(1, 1), (3, 2), (8, 2), (16, 2)])
def test_grid_quad_tiles_shapes(dx, dy):
    print(f"case: grid quads dx={dx} dy={dy} n=300 32x32", flush=True)
    v = workloads.gmm_general(300, dx + dy, seed=150 + dx * 10 + dy)
    hx = workloads.geomspace(0.1, 4.0, 32)
    hy = workloads.geomspace(0.05, 2.0, 32)
    _, tot, pp, nonfin, ref = run_grid(v[:, :dx], v[:, dx:], hx, hy)
    assert nonfin == 0
    check(tot, pp, ref)


def test_grid_tiny_bandwidths_wide_range_and_fixup():
    # Largest terms hundreds to thousands of binary orders below the
    # neighbour shifts: exercises the wide-range kernel values and the exact
    # per-entry recomputation.
    print("case: grid tiny bandwidths", flush=True)
    x, y = workloads.gmm(500, seed=23, dx=2)
    hx = [1e-3, 3e-3, 1e-2, 0.05]
    hy = [1e-3, 4e-3, 0.02]
    _, tot, pp, nonfin, ref = run_grid(x, y, hx, hy)
    assert nonfin == 0
    assert np.min(ref) < -1000.0  # the regime is really extreme
    check(tot, pp, ref)


def test_grid_deterministic_and_reused_shifts():
    print("case: grid determinism", flush=True)
    x, y = workloads.gmm(2000, seed=24, dx=3)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    hx = hy = workloads.geomspace(0.1, 3.0, 12)
    a = m.loo_grid(hx, hy, per_point=True)
    b = m.loo_grid(hx, hy, per_point=True)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    # a second, different grid on the same model reuses the neighbour shifts
    hx2 = workloads.geomspace(0.3, 1.0, 3)
    t2, pp2, _ = m.loo_grid(hx2, [0.2, 0.4], per_point=True)
    ref = oracle.loo_grid(xo, yo, hx2, [0.2, 0.4], nthreads=NT)
    P.assert_points(pp2.cpu().numpy(), ref)


def test_grid_highdim_subset_16x16():
    print("case: highdim subset n=3000 16x16 grid (dx=16, dy=2)", flush=True)
    x, y = workloads.highdim(3000, seed=5)
    hx, hy = workloads.WORKLOADS["highdim"]["grid"]
    _, tot, pp, nonfin, ref = run_grid(x, y, hx, hy)
    assert nonfin == 0
    check(tot, pp, ref)
    # grid argmax agrees with the oracle's
    assert int(np.argmax(tot)) == int(np.argmax(oracle.totals(ref)))


def rerun_classes(x, y, hx, hy, lim=-130.0, margin=8.0):
    """CPU count (FP64, all pairs) of the points the FP32 pass flags for the
    FP64 rerun, by where their flagged cells lie, for ascending grids of one
    16 x 16 tile: the shifted sum of a cell falls as either bandwidth falls,
    so a point has flagged cells iff cell (0, 0) is below 2^lim, and one
    outside the first 4 x 4 cells iff cell (4, 0) or (0, 4) is.  Points
    within 2^margin of the threshold are left out of both counts."""
    x = np.asarray(x, np.float32).astype(np.float64)
    y = np.asarray(y, np.float32).astype(np.float64)
    d2x = ((x[:, None, :] - x[None, :, :]) ** 2).sum(-1)
    d2y = ((y[:, None, :] - y[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2x, np.inf)
    np.fill_diagonal(d2y, np.inf)
    u = d2x - d2x.min(1, keepdims=True)
    v = d2y - d2y.min(1, keepdims=True)

    def log2_sum(a, b):
        t = u * (np.log2(np.e) / (2 * hx[a] ** 2)) + v * (np.log2(np.e) / (2 * hy[b] ** 2))
        mn = t.min(1)
        return -mn + np.log2(np.exp2(-(t - mn[:, None])).sum(1))

    c00, c40, c04 = log2_sum(0, 0), log2_sum(4, 0), log2_sum(0, 4)
    below, above = (lambda z: z < lim - margin), (lambda z: z > lim + margin)
    packed = below(c00) & above(c40) & above(c04)
    full = below(c40) | below(c04)
    return int(packed.sum()), int(full.sum())


def test_grid_packed_and_full_fp64_reruns():
    # Points whose cells the FP32 pass cannot carry are recomputed in FP64:
    # those whose flagged cells all lie in the tile's first 4 x 4 cells four
    # to a product step, the others one per step.  Both kinds are present
    # here (counted on the CPU); every point matches the oracle, and the
    # grouped launch over two ranges gives the one-call totals bit for bit.
    print("case: highdim subset n=2000 16x16, packed and full FP64 reruns", flush=True)
    x, y = workloads.highdim(2000, seed=7)
    hx, hy = workloads.WORKLOADS["highdim"]["grid"]
    packed, full = rerun_classes(x, y, hx, hy)
    print(f"CPU count: {packed} points for the packed rerun, {full} for the full rerun", flush=True)
    assert packed >= 50 and full >= 50
    _, tot, pp, nonfin, ref = run_grid(x, y, hx, hy)
    assert nonfin == 0
    check(tot, pp, ref)
    _, _, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    t = torch.empty(256, dtype=torch.float64, device="cuda")
    cde().launch_batch([(m, 0, 1024, None, None)], hx, hy)
    cde().launch_batch([(m, 1024, 2000, t, None)], hx, hy)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), tot)
    m.close()


@pytest.mark.parametrize("variant", ["valu_fp32", "mfma_bf16x3"])
def test_grid_distance_variants_reported(variant):
    # dx = 16 options that form x-distances approximately (FP32 differences,
    # or a split-bf16 x3 cross term on the matrix cores) in the same pass
    # structure as the default: their error against the oracle is reported,
    # and gated here at the bound measured on this subset; the exact default
    # path on the same model is checked at the parity tolerance.
    print(f"case: highdim subset n=2000 16x16 grid, x-distance variant {variant}", flush=True)
    x, y = workloads.highdim(2000, seed=6)
    hx, hy = workloads.WORKLOADS["highdim"]["grid"]
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    from paper_1206_5278_amd import _binding as B
    xt = {"valu_fp32": B.CDE_XTERM_VALU_F32, "mfma_bf16x3": B.CDE_XTERM_MFMA_BF16X3}[variant]
    tot_x, pp_x, nf = m.loo_grid(hx, hy, per_point=True, xterm=xt)
    tot_v, pp_v, _ = m.loo_grid(hx, hy, per_point=True)
    ref = oracle.loo_grid(xo, yo, hx, hy, nthreads=NT)
    P.assert_points(pp_v.cpu().numpy(), ref)  # exact path unchanged
    assert int(nf.item()) == 0
    ex = pp_x.cpu().numpy()
    err = np.abs(ex - ref) / np.maximum(1.0, np.abs(ref))
    rt = oracle.totals(ref)
    terr = np.abs(tot_x.cpu().numpy() - rt) / np.abs(rt)
    print(f"{variant}: per-point rel err max {err.max():.3e} median {np.median(err):.3e}; "
          f"total rel err max {terr.max():.3e} median {np.median(terr):.3e}", flush=True)
    assert np.all(np.isfinite(ex))
    # measured on this subset: FP32 differences 3.8e-5 per point, 5.5e-8 on
    # totals; bf16 x3 cross term 7.5e-3 and 3.6e-6; bounds at about 2x
    bound = {"valu_fp32": (1e-4, 2e-7), "mfma_bf16x3": (2e-2, 1e-5)}[variant]  # (per point, total)
    assert err.max() <= bound[0] and terr.max() <= bound[1]
