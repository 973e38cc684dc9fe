"""Shared helpers of the GPU parity tests: seeded inputs, device transfer and
the tolerance checks.

Tolerances (FP32 path; FP64 path uses the `f64` variants):
  per point : |l - l*| <= 1e-5 * max(1, |l*|)
  total     : |S - S*| <= 1e-6 * scale, scale = |S*|, or sum_i |l*_i| when
              |S*| < 0.01 * sum_i |l*_i| (a total near zero is a cancellation)
  gradient  : |g_k - g*_k| <= 1e-4 * max(|g*_k|, 1e-2 * max_k |g*_k|)
The oracle always reads the same values the GPU received (FP32 inputs are
promoted exactly to FP64).
"""
import numpy as np
import torch

PER_POINT = 1e-5
TOTAL = 1e-6
GRAD = 1e-4


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def f32_pair(x, y):
    """Round once to FP32; returns (host float64 copies of the FP32 values,
    device FP32 tensors)."""
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    y32 = np.ascontiguousarray(y, dtype=np.float32)
    return (x32.astype(np.float64), y32.astype(np.float64),
            to_dev(x32, torch.float32), to_dev(y32, torch.float32))


def assert_points(got, ref, tol=PER_POINT, what="per-point"):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    err = np.abs(got - ref)
    bound = tol * np.maximum(1.0, np.abs(ref))
    bad = np.flatnonzero(~(err <= bound))
    assert bad.size == 0, (f"{what}: {bad.size} of {err.size} outside tolerance; worst at "
                           f"{int(bad[np.argmax(err[bad] / bound[bad])])}: got "
                           f"{got.flat[bad[0]]!r} ref {ref.flat[bad[0]]!r}")
    return float(np.max(err / np.maximum(1.0, np.abs(ref)))) if err.size else 0.0


def assert_total(got, ref, ref_points, tol=TOTAL):
    scale = abs(ref)
    l1 = float(np.sum(np.abs(ref_points)))
    if scale < 0.01 * l1:
        scale = l1
    err = abs(got - ref)
    assert err <= tol * scale, f"total: got {got!r} ref {ref!r} rel err {err / scale:.3e}"
    return err / scale


def assert_grad(got, ref, tol=GRAD):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    floor = 1e-2 * np.max(np.abs(ref))
    bound = tol * np.maximum(np.abs(ref), floor)
    err = np.abs(got - ref)
    assert np.all(err <= bound), f"gradient: got {got} ref {ref} rel {err / np.maximum(np.abs(ref), floor)}"
    return float(np.max(err / np.maximum(np.abs(ref), floor)))
