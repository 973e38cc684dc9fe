"""GPU check of cde_loo_grad_noalloc, the allocation-free variant of
cde_loo_grad (value and bandwidth gradient of Section 3, eq. 3), called
through the C ABI: two calls in a row, the second on a smaller model, each
against cde_loo_grad on the same model and the FP64 oracle; the size limit
of its static scratch is enforced with CDE_EUNSUPPORTED."""
import ctypes
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


def noalloc_grad(lib, m, h, per_point=True):
    from paper_1206_5278_amd import _binding as B
    total = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty(m.dx + m.dy, dtype=torch.float64, device="cuda")
    pp = torch.empty(m.n, dtype=torch.float64, device="cuda") if per_point else None
    st = lib.cde_loo_grad_noalloc(m.handle, B.doubles(h), B.CDE_COND, total.data_ptr(), grad.data_ptr(),
                                  pp.data_ptr() if pp is not None else None,
                                  torch.cuda.current_stream().cuda_stream)
    B.check(st, "cde_loo_grad_noalloc")
    return total, grad, pp


@pytest.mark.parametrize("n_first,n_second", [(60_000, 3_000), (5_000, 777)])
def test_noalloc_matches_loo_grad_twice(n_first, n_second):
    import paper_1206_5278_amd as cde
    from paper_1206_5278_amd import _binding as B
    lib = B.load()
    for n in (n_first, n_second):
        print(f"case: cde_loo_grad_noalloc photoz n={n}", flush=True)
        x, y = workloads.photoz(n, seed=50 + n)
        xo, yo, xd, yd = P.f32_pair(x, y)
        m = cde.Model(xd, yd)
        h = cde.normal_reference_bandwidths(xo, yo).tolist()
        t_na, g_na, pp_na = noalloc_grad(lib, m, h)
        bytes_before = m.device_bytes
        t_ref, g_ref, pp_ref = m.loo_grad(h, per_point=True)
        torch.cuda.synchronize()
        # against cde_loo_grad at the parity bar (the no-allocation call may
        # split j into fewer chunks, which changes only the rounding) ...
        a, b = pp_na.cpu().numpy(), pp_ref.cpu().numpy()
        P.assert_points(a, b)
        P.assert_total(float(t_na.item()), float(t_ref.item()), b)
        P.assert_grad(g_na.cpu().numpy(), g_ref.cpu().numpy())
        # ... bit for bit where both chunk the same way (small n)
        if n <= 5_000:
            assert torch.equal(t_na, t_ref) and torch.equal(g_na, g_ref) and torch.equal(pp_na, pp_ref)
        # and the oracle's bar on sampled points
        idx = np.sort(np.random.default_rng(n).choice(n, 64, replace=False))
        ell = oracle.loo(xo, yo, h, idx=idx, nthreads=NT)
        P.assert_points(a[idx], ell)
        # the no-allocation call held no model scratch of its own
        assert bytes_before <= B.workspace_bytes(n, 5, 1, B.CDE_F32)
        m.close()


def test_noalloc_beyond_its_scratch_is_rejected():
    import paper_1206_5278_amd as cde
    from paper_1206_5278_amd import _binding as B
    lib = B.load()
    print("case: cde_loo_grad_noalloc size limit, dx=16 dy=2 n=230000", flush=True)
    n = 230_000
    x = torch.randn(n, 16, device="cuda")
    y = torch.randn(n, 2, device="cuda")
    m = cde.Model(x, y)
    with pytest.raises(B.CdeError) as ei:
        noalloc_grad(lib, m, [1.0] * 18, per_point=False)
    assert ei.value.status == B.CDE_EUNSUPPORTED and "64 MiB" in str(ei.value)
    m.close()
