"""ctypes binding of the C ABI in include/cde.h (argument marshalling only).

Every step of the computation runs in the HIP library ``libcde.so``; this
module converts Python/torch arguments into pointers and sizes.  There is no
CPU fallback: if the library is missing the import of the binding fails with
an error that says how to build it.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcde.so")

CDE_OK, CDE_EINVAL, CDE_ENOMEM, CDE_EDEVICE, CDE_EUNSUPPORTED = range(5)
CDE_F32, CDE_F64 = 0, 1
CDE_COND, CDE_JOINT = 0, 1
CDE_XTERM_AUTO, CDE_XTERM_VALU, CDE_XTERM_MFMA_BF16X3, CDE_XTERM_VALU_F32 = 0, 1, 2, 3
CDE_GAUSSIAN, CDE_EPANECHNIKOV = 0, 1
ABI_VERSION = 4

# Every symbol the header declares, with (restype, argtypes).
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_i32, _i64 = ctypes.c_int32, ctypes.c_int64
SIGNATURES = {
    "cde_abi_version": (ctypes.c_int, []),
    "cde_last_error": (ctypes.c_char_p, []),
    "cde_create": (ctypes.c_int, [ctypes.POINTER(_vp), _vp, _vp, _i64, _i32, _i32, ctypes.c_int, _vp]),
    "cde_destroy": (ctypes.c_int, [_vp]),
    "cde_model_device_bytes": (ctypes.c_size_t, [_vp]),
    "cde_workspace_bytes": (ctypes.c_size_t, [_i64, _i32, _i32, ctypes.c_int, _i32, _i32]),
    "cde_loo_loglik": (ctypes.c_int, [_vp, _dp, _i32, _dp, _i32, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, _vp, _vp, _vp, _vp]),
    "cde_loo_loglik_list": (ctypes.c_int, [_vp, _dp, _i32, ctypes.c_int, ctypes.c_int, _vp, _vp,
                                           _vp]),
    "cde_loo_grad": (ctypes.c_int, [_vp, _dp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "cde_density_query": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _dp, ctypes.c_int, _vp, _vp]),
    "cde_conditional_mean": (ctypes.c_int, [_vp, _vp, _i64, _dp, _vp, _vp]),
    "cde_density_summary": (ctypes.c_int, [_vp, _vp, _i64, _i64, ctypes.c_double, _vp, _vp]),
    "cde_cv_ise": (ctypes.c_int, [_vp, _dp, _vp, _vp, _vp]),
    "cde_check_bandwidths": (ctypes.c_int, [_dp, _i32, _i32, _dp, ctypes.c_int, _i32]),
    "cde_loo_grad_noalloc": (ctypes.c_int, [_vp, _dp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "cde_launch_batch": (ctypes.c_int, [_vp, _i32, _dp, _i32, _dp, _i32, ctypes.c_int, _vp]),
    "cde_batch_round_points": (ctypes.c_int64, [_i32, _i32]),
}


class WorkItem(ctypes.Structure):
    """cde_work_item of include/cde.h: points [i0, i1) of one model."""
    _fields_ = [("model", ctypes.c_void_p), ("i0", ctypes.c_int64), ("i1", ctypes.c_int64),
                ("totals_dev", ctypes.c_void_p), ("n_nonfinite_dev", ctypes.c_void_p)]


class CdeError(RuntimeError):
    """A non-OK status from the C ABI."""

    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: status {status}: {message}")


_lib = None


def load(path: str = LIB_PATH):
    """Load ``libcde.so`` and declare the signatures (cached)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"HIP library not found at {path}; build it with "
            "`python -m paper_1206_5278_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path == LIB_PATH:
        _lib = lib
    return lib


def check(status: int, where: str) -> None:
    if status != CDE_OK:
        msg = load().cde_last_error()
        raise CdeError(status, where, msg.decode() if msg else "")


def doubles(values) -> ctypes.Array:
    vals = [float(v) for v in values]
    return (ctypes.c_double * max(1, len(vals)))(*vals)


def workspace_bytes(n: int, dx: int, dy: int, precision: int = CDE_F32, n_hx: int = 0,
                    n_hy: int = 0) -> int:
    """Device bytes of a model of this shape after one n_hx x n_hy grid call
    (``cde_workspace_bytes``); 0 for shapes the library rejects."""
    return int(load().cde_workspace_bytes(int(n), int(dx), int(dy), int(precision), int(n_hx),
                                          int(n_hy)))
