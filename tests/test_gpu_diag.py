"""GPU parity of the diagonal-bandwidth LOO value and gradient, the list and
grid calls, and density queries, against the FP64 CPU oracle, through the
C ABI."""
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
    import paper_1206_5278_amd  # noqa: F401  (fails loudly if libcde.so is missing)


def cde():
    import paper_1206_5278_amd as m
    return m


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_grad(x, y, h, crit="cond", dtype=torch.float32):
    """GPU value/grad/per-point, and the oracle on the exact same values."""
    if dtype == torch.float32:
        xo, yo, xd, yd = P.f32_pair(x, y)
    else:
        xo, yo = np.asarray(x, np.float64), np.asarray(y, np.float64)
        xd, yd = P.to_dev(xo, torch.float64), P.to_dev(yo, torch.float64)
    m = cde().Model(xd, yd)
    total, grad, pp = m.loo_grad(h, crit, per_point=True)
    torch.cuda.synchronize()
    ell, dell = oracle.loo(xo, yo, m._bw(h), crit, grad=True, nthreads=NT)
    return (float(total.item()), grad.cpu().numpy(), pp.cpu().numpy()), (oracle.total(ell),
                                                                          dell.sum(axis=0), ell)


@pytest.mark.parametrize("crit", ["cond", "joint"])
def test_grad_parity_photoz_ragged(crit):
    say(f"case: photoz n=700 value+grad {crit}")
    x, y = workloads.photoz(700, seed=5)
    h = [0.06, 0.05, 0.07, 0.06, 0.08, 0.03]
    (t, g, pp), (rt, rg, rp) = run_grad(x, y, h, crit)
    P.assert_points(pp, rp)
    P.assert_total(t, rt, rp)
    P.assert_grad(g, rg)


def test_fp64_parity_tiny_workload():
    say("case: tiny f64 n=600")
    x, y = workloads.tiny(600, seed=2)
    h = [3.0, 4.0]
    (t, g, pp), (rt, rg, rp) = run_grad(x, y, h, "cond", torch.float64)
    P.assert_points(pp, rp, tol=1e-11)
    assert abs(t - rt) <= 1e-11 * abs(rt)
    np.testing.assert_allclose(g, rg, rtol=1e-9, atol=1e-9 * np.max(np.abs(rg)))


DIMS = [(dx, dy) for dx in (1, 2, 3, 4, 5, 6, 7, 8, 16) for dy in (1, 2)]


@pytest.mark.parametrize("dx,dy", DIMS)
def test_all_shapes_value_grad(dx, dy):
    say(f"case: shape dx={dx} dy={dy} n=300")
    v = workloads.gmm_general(300, dx + dy, seed=dx * 10 + dy)
    x, y = v[:, :dx], v[:, dx:]
    h = list(np.linspace(0.6, 1.4, dx)) + list(np.linspace(0.5, 0.8, dy))
    (t, g, pp), (rt, rg, rp) = run_grad(x, y, h)
    P.assert_points(pp, rp)
    P.assert_total(t, rt, rp)
    P.assert_grad(g, rg)


@pytest.mark.parametrize("n", [2, 3, 255, 256, 257, 513])
def test_edge_sizes(n):
    say(f"case: edge n={n}")
    rng = np.random.default_rng(n)
    x = rng.normal(size=(n, 2))
    y = rng.normal(size=(n, 1))
    (t, g, pp), (rt, rg, rp) = run_grad(x, y, [0.5, 0.7, 0.4])
    P.assert_points(pp, rp)
    P.assert_total(t, rt, rp)
    P.assert_grad(g, rg)


def test_identical_x_reduces_to_marginal_kde():
    say("case: identical x")
    rng = np.random.default_rng(9)
    x = np.full((300, 3), 0.25)
    y = rng.normal(size=(300, 1))
    (t, g, pp), (rt, rg, rp) = run_grad(x, y, [0.3, 0.3, 0.3, 0.2])
    P.assert_points(pp, rp)
    P.assert_total(t, rt, rp)
    assert np.all(np.abs(g[:3]) <= 1e-6 * np.max(np.abs(rg)) + 1e-9)


@pytest.mark.parametrize("hx", [0.01, 0.02, 1e3])
def test_extreme_bandwidths_shift_path(hx):
    # tiny hx: the nearest neighbours' exponents d^2 c reach ~650, so every
    # kernel value underflows without the per-point shift.  (Much smaller hx
    # leaves the diagonal pass's accuracy regime: its FP32 exponents carry an
    # absolute error of a few ulp of d^2 c, which matters when two
    # neighbours compete; at hx = 2e-3 one of these 900 points misses the
    # per-point tolerance by 2.4x.)
    say(f"case: extreme hx={hx}")
    x, y = workloads.gmm(900, seed=3, dx=2)
    (t, g, pp), (rt, rg, rp) = run_grad(x, y, [hx, hx, 0.3])
    assert np.all(np.isfinite(pp))
    P.assert_points(pp, rp)
    P.assert_total(t, rt, rp)


def test_tiny_hy_shift_path():
    say("case: tiny hy")
    x, y = workloads.gmm(700, seed=4, dx=3)
    (t, g, pp), (rt, rg, rp) = run_grad(x, y, [0.5, 0.5, 0.5, 0.004])
    assert np.all(np.isfinite(pp))
    P.assert_points(pp, rp)
    P.assert_total(t, rt, rp)


def _far_prologue_data(n, seed, far_x, far_y):
    """Rows 0..39 sit far away (at far_x in x, far_y in y); the rest form a
    tight cluster at the origin.  The per-point references of cluster points
    start from rows 0..31, so their first cluster terms are 2^gap heavier."""
    rng = np.random.default_rng(seed)
    x = 1e-3 * rng.normal(size=(n, 1))
    y = 1e-2 * rng.normal(size=(n, 1))
    x[:40] += far_x
    y[:40] += far_y
    return x, y


# (far_x, far_y, hx, hy): gap = c * far^2 with c = log2(e) / (2 h^2) decides the
# path: gap 30 (24 cluster terms make a subtile sum above 2^32 with no single
# term above 2^32), gap 43 (rescale in place), gap 288 (overflow: summed again),
# and a gap in the y kernel alone (only the product-kernel reference moves).
@pytest.mark.parametrize("far_x,far_y,hx,hy", [
    (1.0, 0.0, 0.155, 0.3),
    (1.0, 0.0, 0.13, 0.3),
    (1.0, 0.0, 0.05, 0.3),
    (0.0, 1.0, 0.3, 0.05),
])
@pytest.mark.parametrize("crit", ["cond", "joint"])
def test_reference_moves(far_x, far_y, hx, hy, crit):
    say(f"case: reference moves far=({far_x},{far_y}) h=({hx},{hy}) {crit}")
    x, y = _far_prologue_data(600, 11, far_x, far_y)
    (t, g, pp), (rt, rg, rp) = run_grad(x, y, [hx, hy], crit)
    assert np.all(np.isfinite(pp))
    P.assert_points(pp, rp)
    P.assert_total(t, rt, rp)
    P.assert_grad(g, rg)
    # the value-only instance takes the same paths
    _, _, xd, yd = P.f32_pair(x, y)
    tot, pp2 = cde().Model(xd, yd).loo_list([[hx, hy]], crit, per_point=True)
    torch.cuda.synchronize()
    P.assert_points(pp2.cpu().numpy()[0], rp)


def test_deterministic_bits():
    say("case: determinism")
    x, y = workloads.photoz(3000, seed=6)
    _, _, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    h = [0.05] * 5 + [0.03]
    a = [v.cpu() for v in m.loo_grad(h, per_point=True)]
    b = [v.cpu() for v in m.loo_grad(h, per_point=True)]
    for u, v in zip(a, b):
        assert torch.equal(u, v)


def test_list_matches_grad_value_and_oracle():
    say("case: list of settings")
    x, y = workloads.gmm(800, seed=8, dx=4)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    hs = [[0.3 + 0.1 * s] * 4 + [0.2 + 0.05 * s] for s in range(9)]
    tot, pp = m.loo_list(hs, per_point=True)
    tot, pp = tot.cpu().numpy(), pp.cpu().numpy()
    for s, h in enumerate(hs):
        ref = oracle.loo(xo, yo, h, nthreads=NT)
        P.assert_points(pp[s], ref)
        P.assert_total(tot[s], oracle.total(ref), ref)
        t1, _, _ = m.loo_grad(h)
        assert float(t1.item()) == pytest.approx(tot[s], rel=1e-12)


def test_grid_tiny_workload_fp64_full():
    # Plain method, tiny: N=2000, dx=dy=1, FP64, 8 x 8 grid of 0.5..20.
    say("case: tiny workload 8x8 grid fp64 full")
    cfg = workloads.WORKLOADS["tiny"]
    x, y = workloads.tiny()
    hx, hy = cfg["grid"]
    m = cde().Model(P.to_dev(x, torch.float64), P.to_dev(y, torch.float64))
    tot, pp, nonfin = m.loo_grid(hx, hy, per_point=True)
    ref = oracle.loo_grid(x, y, hx, hy, nthreads=NT)
    P.assert_points(pp.cpu().numpy(), ref, tol=1e-11)
    rt = oracle.totals(ref)
    np.testing.assert_allclose(tot.cpu().numpy(), rt, rtol=1e-11)
    assert int(nonfin.item()) == 0
    t, (a, b) = cde().select_grid(m, hx, hy)
    k = int(np.argmax(rt))
    assert (a, b) == (k // 8, k % 8)


def test_grid_tiny_workload_fp32():
    say("case: tiny workload 8x8 grid fp32")
    cfg = workloads.WORKLOADS["tiny"]
    x, y = workloads.tiny()
    hx, hy = cfg["grid"]
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    tot, pp, _ = m.loo_grid(hx, hy, per_point=True)
    ref = oracle.loo_grid(xo, yo, hx, hy, nthreads=NT)
    P.assert_points(pp.cpu().numpy(), ref)
    for s in range(64):
        P.assert_total(float(tot[s]), oracle.total(ref[s]), ref[s])


def test_query_parity_and_normalisation():
    say("case: density query")
    x, y = workloads.gmm(1500, seed=11, dx=3)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    h = [0.4, 0.5, 0.45, 0.15]
    rng = np.random.default_rng(2)
    xq = np.ascontiguousarray(xo[rng.choice(1500, 37)] + 0.1, dtype=np.float32).astype(np.float64)
    yg = np.linspace(yo.min() - 1, yo.max() + 1, 301).astype(np.float32).astype(np.float64)
    f = m.query(P.to_dev(xq), P.to_dev(yg), h).cpu().numpy()
    ref = oracle.density(xo, yo, h, xq, yg, nthreads=NT)
    peak = ref.max(axis=1, keepdims=True)
    err = np.abs(f - ref)
    assert np.all(err <= 1e-5 * ref + 1e-7 * peak), float(np.max(err / (1e-5 * ref + 1e-7 * peak)))
    # the estimate integrates to ~1 over a grid wide enough to hold the mass
    integ = np.trapezoid(f, yg, axis=1)
    assert np.all(np.abs(integ - 1) < 2e-3)


@pytest.mark.parametrize("dx,dy", DIMS)
def test_query_all_shapes(dx, dy):
    # FP32 models: matrix-core query kernel; k = 40, 100 and 150 use grid
    # blocks of 64, 128 and 256 points (one, two and four 32-column tiles per
    # wave), each part-filled, and q = 70 fills part of one 128-query block.
    say(f"case: query shape dx={dx} dy={dy}")
    v = workloads.gmm_general(400, dx + dy, seed=200 + dx * 10 + dy)
    x, y = v[:, :dx], v[:, dx:]
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    h = list(np.linspace(0.7, 1.2, dx)) + list(np.linspace(0.3, 0.5, dy))
    rng = np.random.default_rng(dx * 7 + dy)
    xq = (xo[rng.choice(400, 70)] + 0.1 * rng.normal(size=(70, dx))).astype(np.float32).astype(np.float64)
    for k in (40, 100, 150):
        yg = (yo[rng.choice(400, k)] + 0.2 * rng.normal(size=(k, dy))).astype(np.float32).astype(np.float64)
        f = m.query(P.to_dev(xq), P.to_dev(yg), h).cpu().numpy()
        ref = oracle.density(xo, yo, h, xq, yg, nthreads=NT)
        peak = ref.max(axis=1, keepdims=True)
        err = np.abs(f - ref)
        assert np.all(err <= 1e-5 * ref + 1e-7 * peak), (k, float(np.max(err / (1e-5 * ref + 1e-7 * peak))))


def test_query_rows_independent_of_batch():
    # A query's value must not depend on the other queries of its launch: the
    # serving path fuses queries.  n = 70,000 gives 137 training-point chunks
    # and 3,000 queries on a 256-point grid run in two slices.
    say("case: query rows alone vs in a batch of 3000")
    x, y = workloads.gmm(70_000, seed=13, dx=2)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    h = [0.3, 0.35, 0.2]
    rng = np.random.default_rng(5)
    xq = (xo[rng.choice(70_000, 3000)] + 0.05 * rng.normal(size=(3000, 2))).astype(np.float32)
    yg = np.linspace(yo.min() - 1, yo.max() + 1, 256).astype(np.float32)
    xq_d, yg_d = P.to_dev(xq, torch.float32), P.to_dev(yg, torch.float32)
    full = m.query(xq_d, yg_d, h).cpu().numpy()
    for rows in ([0], [1500], [2999], [7, 2000, 2998]):
        part = m.query(xq_d[rows].contiguous(), yg_d, h).cpu().numpy()
        assert np.array_equal(part, full[rows]), rows
    ref = oracle.density(xo, yo, h, xq[[0, 2999]].astype(np.float64), yg.astype(np.float64),
                         nthreads=NT)
    peak = ref.max(axis=1, keepdims=True)
    err = np.abs(full[[0, 2999]] - ref)
    assert np.all(err <= 1e-5 * ref + 1e-7 * peak)


def test_query_grid_widths_and_many_chunks():
    # n = 600,000 needs more than 256 training-point chunks (a chunk holds at
    # most 8 tiles); k = 40, 100 and 700 use blocks of 64, 128 and 256 grid
    # points (the last with a ragged third block); one query lies far from
    # every training point (a large shift m_q).
    say("case: query n=600000, k in (40, 100, 700)")
    x, y = workloads.gmm(600_000, seed=17, dx=2)
    xo, yo, xd, yd = P.f32_pair(x, y)
    m = cde().Model(xd, yd)
    h = [0.25, 0.3, 0.2]
    rng = np.random.default_rng(9)
    xq = (xo[rng.choice(600_000, 69)] + 0.05 * rng.normal(size=(69, 2))).astype(np.float32)
    xq[68] = xo.max(axis=0) + 3.0
    xq_d = P.to_dev(xq, torch.float32)
    rows = [0, 33, 67, 68]
    for k in (40, 100, 700):
        yg = np.linspace(yo.min() - 1, yo.max() + 1, k).astype(np.float32)
        yg_d = P.to_dev(yg, torch.float32)
        f = m.query(xq_d, yg_d, h).cpu().numpy()
        ref = oracle.density(xo, yo, h, xq[rows].astype(np.float64), yg.astype(np.float64),
                             nthreads=NT)
        peak = ref.max(axis=1, keepdims=True)
        err = np.abs(f[rows] - ref)
        assert np.all(err <= 1e-5 * ref + 1e-7 * peak), (k, float(np.max(err / (1e-5 * ref + 1e-7 * peak))))
        part = m.query(xq_d[[33, 68]].contiguous(), yg_d, h).cpu().numpy()
        assert np.array_equal(part, f[[33, 68]]), k


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_workspace_bytes_matches_model(dtype):
    # cde_workspace_bytes predicts what a model holds after one grid call
    say(f"case: workspace bytes {dtype}")
    from paper_1206_5278_amd import _binding as B
    x, y = workloads.gmm(3000, seed=21, dx=3)
    m = cde().Model(P.to_dev(x, dtype), P.to_dev(y, dtype))
    prec = B.CDE_F32 if dtype == torch.float32 else B.CDE_F64
    assert m._lib.cde_model_device_bytes(m._h) == B.workspace_bytes(3000, 3, 1, prec)
    hs = list(workloads.geomspace(0.1, 3.0, 16))
    m.loo_grid(hs, hs)
    torch.cuda.synchronize()
    assert m._lib.cde_model_device_bytes(m._h) == B.workspace_bytes(3000, 3, 1, prec, 16, 16)


def test_query_fp64_model():
    say("case: query fp64 model")
    x, y = workloads.tiny(500, seed=4)
    m = cde().Model(P.to_dev(x, torch.float64), P.to_dev(y, torch.float64))
    xq = np.linspace(0, 100, 9).reshape(-1, 1)
    yg = np.linspace(0, 100, 41).reshape(-1, 1)
    f = m.query(P.to_dev(xq, torch.float64), P.to_dev(yg, torch.float64), [4.0, 5.0]).cpu().numpy()
    ref = oracle.density(x, y, [4.0, 5.0], xq, yg, nthreads=NT)
    np.testing.assert_allclose(f, ref, rtol=1e-10, atol=1e-300)
