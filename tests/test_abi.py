"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad arguments with status codes before touching
a device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cde.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cde_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1206_5278_amd import _binding
    return _binding.load()


def test_header_declares_expected_calls():
    names = declared_functions()
    for n in ("cde_create", "cde_destroy", "cde_loo_loglik", "cde_loo_grad", "cde_density_query",
              "cde_loo_loglik_list", "cde_last_error", "cde_abi_version", "cde_conditional_mean",
              "cde_density_summary", "cde_cv_ise"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1206_5278_amd import _binding
    out = subprocess.run(["nm", "-D", "--defined-only", _binding.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (cde_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(declared_functions()) <= set(_binding.SIGNATURES)


def test_abi_version(lib):
    assert lib.cde_abi_version() == 4


def test_invalid_arguments_return_status(lib):
    from paper_1206_5278_amd import _binding as B
    h = ctypes.c_void_p()
    assert lib.cde_create(None, 1, 1, 10, 1, 1, 0, None) == B.CDE_EINVAL
    assert lib.cde_create(ctypes.byref(h), None, None, 10, 1, 1, 0, None) == B.CDE_EINVAL
    assert lib.cde_create(ctypes.byref(h), 8, 8, 1, 1, 1, 0, None) == B.CDE_EINVAL  # n < 2
    assert lib.cde_create(ctypes.byref(h), 8, 8, 10, 0, 1, 0, None) == B.CDE_EINVAL
    assert lib.cde_create(ctypes.byref(h), 8, 8, 10, 65, 1, 0, None) == B.CDE_EUNSUPPORTED
    assert lib.cde_create(ctypes.byref(h), 8, 8, 10, 1, 1, 7, None) == B.CDE_EINVAL
    assert b"precision" in lib.cde_last_error()
    hv = B.doubles([1.0, 1.0])
    assert lib.cde_loo_grad(None, hv, 0, 8, 8, None, None) == B.CDE_EINVAL
    assert lib.cde_loo_loglik(None, hv, 1, hv, 1, 0, 0, 0, 8, None, None, None) == B.CDE_EINVAL
    assert lib.cde_loo_loglik_list(None, hv, 1, 0, 0, 8, None, None) == B.CDE_EINVAL
    assert lib.cde_density_query(None, 8, 1, 8, 1, hv, 0, 8, None) == B.CDE_EINVAL
    assert lib.cde_cv_ise(None, hv, 8, None, None) == B.CDE_EINVAL
    assert lib.cde_loo_grad_noalloc(None, hv, 0, 8, 8, None, None) == B.CDE_EINVAL
    assert lib.cde_launch_batch(None, 1, hv, 1, hv, 1, 0, None) == B.CDE_EINVAL
    items = (B.WorkItem * 1)()
    assert lib.cde_launch_batch(ctypes.cast(items, ctypes.c_void_p), 1, hv, 17, hv, 1, 0, None) == B.CDE_EINVAL
    assert b"[1, 16]" in lib.cde_last_error()
    assert lib.cde_launch_batch(ctypes.cast(items, ctypes.c_void_p), 1, hv, 1, hv, 1, 0, None) == B.CDE_EINVAL
    assert b"no model" in lib.cde_last_error()
    assert lib.cde_destroy(None) == B.CDE_OK
    assert lib.cde_model_device_bytes(None) == 0


def test_product_path_does_not_reference_oracle():
    pkg = os.path.join(ROOT, "paper_1206_5278_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "cde_oracle" not in text and "oracle_loo" not in text, f


def test_workspace_bytes_host_arithmetic(lib):
    from paper_1206_5278_amd import _binding as B
    # after cde_create alone: the packed [npad][stride] rows (stride = dx + dy
    # rounded up to 4), 256-byte aligned, and the 512-byte data-extent record
    assert B.workspace_bytes(1000, 5, 1, B.CDE_F32) == 1024 * 8 * 4 + 512
    assert B.workspace_bytes(1000, 5, 1, B.CDE_F64) == 1024 * 8 * 8 + 512
    assert B.workspace_bytes(256, 16, 2, B.CDE_F32) == 256 * 20 * 4 + 512
    # a grid call adds shifts and scratch, growing with the grid
    base = B.workspace_bytes(5000, 3, 1, B.CDE_F32)
    g8 = B.workspace_bytes(5000, 3, 1, B.CDE_F32, 8, 8)
    g16 = B.workspace_bytes(5000, 3, 1, B.CDE_F32, 16, 16)
    assert base < g8 < g16
    # rejected shapes and grid sizes give 0
    for args in [(1, 1, 1, 0), (100, 0, 1, 0), (100, 9, 1, 0), (100, 1, 3, 0), (100, 1, 1, 7),
                 (100, 1, 1, 0, 65, 1), (100, 1, 1, 0, 4, 0), (100, 1, 1, 0, -1, -1)]:
        assert B.workspace_bytes(*args) == 0, args


def test_batch_round_points_unsupported_shapes(lib):
    # shapes the kernels are not built for answer 0 before any device query
    for dx, dy in [(0, 1), (3, 3), (9, 1), (17, 1), (5, 0)]:
        assert lib.cde_batch_round_points(dx, dy) == 0, (dx, dy)


def test_bandwidth_range_check_host(lib):
    """The representable-range rule of the model calls, on the host: each
    c_k = log2(e)/(2 h_k^2) <= 2^59 and X, Y = sum_k range_k^2 c_k <= 2^100
    per axis (FP32 models; 2^900 for all on FP64 models); on the diagonal
    pass also (X + Y)(dx + dy + 2) <= 2^29 (FP32; 2^61 on FP64 models)."""
    import math

    from paper_1206_5278_amd import _binding as B

    def check(rng, h, prec=B.CDE_F32, dx=5, dy=1, diag=0):
        return lib.cde_check_bandwidths(B.doubles(rng), dx, dy, B.doubles(h), prec, diag)

    # the diagonal-pass rule: with range 1 in every dimension and one h,
    # X + Y = 6 c and (X + Y) * 8 <= 2^29 means c <= 2^26 / 6
    hd = math.sqrt(math.log2(math.e) / (2.0 * 2.0 ** 26 / 6.0))
    one = [1.0] * 6
    assert check(one, [hd * (1 + 1e-9)] * 6, diag=1) == B.CDE_OK
    assert check(one, [hd * (1 - 1e-9)] * 6, diag=1) == B.CDE_EUNSUPPORTED
    assert b"diagonal pass" in lib.cde_last_error()
    assert check(one, [hd * (1 - 1e-9)] * 6, diag=0) == B.CDE_OK  # the grid pass takes it
    assert check(one, [hd * 1e-3] * 6, B.CDE_F64, diag=1) == B.CDE_OK

    one = [1.0] * 6
    assert check(one, [0.1] * 6) == B.CDE_OK
    # the coefficient bound: c = 2^59 exactly at h* = sqrt(log2(e) / 2^60)
    hstar = math.sqrt(math.log2(math.e) / 2.0 ** 60)
    assert check([0.0] * 6, [0.1] * 5 + [hstar * (1 + 1e-9)]) == B.CDE_OK
    assert check([0.0] * 6, [0.1] * 5 + [hstar * (1 - 1e-9)]) == B.CDE_EUNSUPPORTED
    assert b"y bandwidth" in lib.cde_last_error()
    assert check([0.0] * 6, [hstar * 0.5] + [0.1] * 5) == B.CDE_EUNSUPPORTED
    assert b"x bandwidth" in lib.cde_last_error()
    # the data-relative bound: the largest exponent sum_k range_k^2 c_k
    big = [1e20, 1.0, 1.0, 1.0, 1.0, 1.0]
    assert check(big, [1.0] * 6) == B.CDE_EUNSUPPORTED
    assert check(big, [1e6] + [1.0] * 5) == B.CDE_OK
    # the same settings on FP64 models, whose bounds are 2^900
    assert check(big, [1.0] * 6, B.CDE_F64) == B.CDE_OK
    assert check(one, [1e-100] * 6, B.CDE_F64) == B.CDE_OK
    assert check(one, [1e-140] * 6, B.CDE_F64) == B.CDE_EUNSUPPORTED
    # malformed arguments
    assert check(one, [0.1] * 5 + [0.0]) == B.CDE_EINVAL
    assert check(one, [0.1] * 5 + [float("nan")]) == B.CDE_EINVAL
    assert check([1.0] * 5 + [-1.0], [0.1] * 6) == B.CDE_EINVAL
    assert check([1.0] * 5 + [float("inf")], [0.1] * 6) == B.CDE_EINVAL
    assert check(one, [0.1] * 6, 7) == B.CDE_EINVAL
    assert lib.cde_check_bandwidths(None, 5, 1, B.doubles([0.1] * 6), 0, 0) == B.CDE_EINVAL
    assert check(one, [0.1] * 6, B.CDE_F32, 0, 1) == B.CDE_EINVAL
