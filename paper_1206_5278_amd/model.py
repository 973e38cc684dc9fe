"""Python face of the library: a resident training set and the calls of the
C ABI on it.  torch supplies device memory and streams only; every step of the
computation runs in ``libcde.so``.

Method: Holmes, Gray & Isbell, "Fast Nonparametric Conditional Density
Estimation" -- eq. (1) (the double-kernel estimator) and eq. (3) with the
A_i expansion of Section 3.2 (the leave-one-out likelihood).  hx is the
x-bandwidth (the paper's h2) and hy the y-bandwidth (the paper's h1).
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import _binding as B

CRITERIA = {"cond": B.CDE_COND, "conditional": B.CDE_COND, "joint": B.CDE_JOINT}
KERNELS = {"gaussian": B.CDE_GAUSSIAN, "epanechnikov": B.CDE_EPANECHNIKOV}


def _stream_ptr(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Model:
    """A training set {(x_i, y_i)} resident in the model's own device memory.

    x: [n, dx] and y: [n, dy] CUDA tensors of float32 (FP32 path) or float64
    (FP64 path).  The values handed in are the dataset; they are copied and
    packed on the current stream, after which the inputs may be released."""

    def __init__(self, x: torch.Tensor, y: torch.Tensor, stream=None):
        if not (x.is_cuda and y.is_cuda):
            raise ValueError("x and y must be CUDA (HIP) tensors")
        if x.dtype != y.dtype or x.dtype not in (torch.float32, torch.float64):
            raise ValueError("x and y must both be float32 or both float64")
        if y.dim() == 1:
            y = y.reshape(-1, 1)
        if x.dim() == 1:
            x = x.reshape(-1, 1)
        if x.shape[0] != y.shape[0]:
            raise ValueError("x and y must have the same number of rows")
        self._lib = B.load()
        x = x.contiguous()
        y = y.contiguous()
        self.n, self.dx = int(x.shape[0]), int(x.shape[1])
        self.dy = int(y.shape[1])
        self.dtype = x.dtype
        self.device = x.device
        self.precision = B.CDE_F64 if x.dtype == torch.float64 else B.CDE_F32
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            st = self._lib.cde_create(ctypes.byref(h), x.data_ptr(), y.data_ptr(), self.n, self.dx,
                                      self.dy, self.precision, _stream_ptr(stream))
        B.check(st, "cde_create")
        self._h = h
        self._keep = (x, y)  # inputs stay alive until the pack has run
        self._keep_stream = stream

    # ------------------------------------------------------------------ utils
    @property
    def handle(self) -> int:
        return self._h.value

    @property
    def device_bytes(self) -> int:
        return int(self._lib.cde_model_device_bytes(self._h))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            B.check(self._lib.cde_destroy(self._h), "cde_destroy")
            self._h = ctypes.c_void_p()
        self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bw(self, h) -> list:
        h = [float(v) for v in (h.tolist() if torch.is_tensor(h) else h)]
        p = self.dx + self.dy
        if len(h) == 2 and p != 2:
            h = [h[0]] * self.dx + [h[1]] * self.dy
        if len(h) != p:
            raise ValueError(f"expected {p} bandwidths (dx+dy) or a pair (hx, hy)")
        return h

    # ------------------------------------------------------------- the calls
    def loo_grid(self, hx, hy, criterion: str = "cond", per_point: bool = False,
                 stream=None, out=None, xterm: int = B.CDE_XTERM_AUTO, kernel: str = "gaussian"):
        """Exact LOO log-likelihood totals over the scalar grid hx x hy
        (kernel "gaussian" or "epanechnikov").

        Returns (totals [len(hx)*len(hy)] float64 on the device, hx-major;
        per-point [G, n] or None; non-finite count tensor [1] int64)."""
        hx = [float(v) for v in hx]
        hy = [float(v) for v in hy]
        g = len(hx) * len(hy)
        totals = out if out is not None else torch.empty(g, dtype=torch.float64, device=self.device)
        pp = torch.empty((g, self.n), dtype=torch.float64, device=self.device) if per_point else None
        nonfin = torch.empty(1, dtype=torch.int64, device=self.device)
        st = self._lib.cde_loo_loglik(self._h, B.doubles(hx), len(hx), B.doubles(hy), len(hy),
                                      CRITERIA[criterion], KERNELS[kernel], int(xterm),
                                      totals.data_ptr(),
                                      pp.data_ptr() if pp is not None else None, nonfin.data_ptr(),
                                      _stream_ptr(stream))
        B.check(st, "cde_loo_loglik")
        return totals, pp, nonfin

    def loo_list(self, hs, criterion: str = "cond", per_point: bool = False, stream=None,
                 kernel: str = "gaussian"):
        """Totals for a list of diagonal settings hs [g][dx+dy] (or pairs), with
        the Gaussian or the Epanechnikov kernel."""
        rows = [self._bw(h) for h in hs]
        flat = [v for r in rows for v in r]
        totals = torch.empty(len(rows), dtype=torch.float64, device=self.device)
        pp = torch.empty((len(rows), self.n), dtype=torch.float64, device=self.device) if per_point else None
        st = self._lib.cde_loo_loglik_list(self._h, B.doubles(flat), len(rows), CRITERIA[criterion],
                                           KERNELS[kernel], totals.data_ptr(),
                                           pp.data_ptr() if pp is not None else None,
                                           _stream_ptr(stream))
        B.check(st, "cde_loo_loglik_list")
        return totals, pp

    def loo_grad(self, h, criterion: str = "cond", per_point: bool = False, stream=None):
        """Value S(h) and dS/dh for one diagonal setting.

        Returns (total [1], grad [dx+dy], per-point [n] or None), float64 on
        the device."""
        hv = self._bw(h)
        total = torch.empty(1, dtype=torch.float64, device=self.device)
        grad = torch.empty(self.dx + self.dy, dtype=torch.float64, device=self.device)
        pp = torch.empty(self.n, dtype=torch.float64, device=self.device) if per_point else None
        st = self._lib.cde_loo_grad(self._h, B.doubles(hv), CRITERIA[criterion], total.data_ptr(),
                                    grad.data_ptr(), pp.data_ptr() if pp is not None else None,
                                    _stream_ptr(stream))
        B.check(st, "cde_loo_grad")
        return total, grad, pp

    def conditional_mean(self, xq: torch.Tensor, h, stream=None) -> torch.Tensor:
        """E[y | xq] (mean of eq. (1)'s density, Gaussian kernel): [q, dy] float64."""
        xq = xq.reshape(-1, self.dx).to(self.dtype).contiguous()
        q = int(xq.shape[0])
        out = torch.empty((q, self.dy), dtype=torch.float64, device=self.device)
        st = self._lib.cde_conditional_mean(self._h, xq.data_ptr(), q, B.doubles(self._bw(h)),
                                            out.data_ptr(), _stream_ptr(stream))
        B.check(st, "cde_conditional_mean")
        return out

    def cv_ise(self, h, terms: bool = False, stream=None):
        """Cross-validated ISE of Section 3 (eq. 2) for one diagonal setting h
        (Gaussian kernels, FP32 models): returns a float64 device tensor
        [ISE, mean T1, mean T2] and, when ``terms``, the per-point [n, 2]
        tensor (T1_i, T2_i) as well.  O(n^3) work."""
        out = torch.empty(3, dtype=torch.float64, device=self.device)
        tm = torch.empty((self.n, 2), dtype=torch.float64, device=self.device) if terms else None
        st = self._lib.cde_cv_ise(self._h, B.doubles(self._bw(h)), out.data_ptr(),
                                  tm.data_ptr() if tm is not None else None, _stream_ptr(stream))
        B.check(st, "cde_cv_ise")
        return (out, tm) if terms else out

    def query(self, xq: torch.Tensor, ygrid: torch.Tensor, h, stream=None, out=None,
              kernel: str = "gaussian"):
        """f(ygrid[g] | xq[q]) of eq. (1) over all training points: [q, k] float64
        (``kernel``: "gaussian", or "epanechnikov" for FP32 models)."""
        xq = xq.reshape(-1, self.dx).to(self.dtype).contiguous()
        ygrid = ygrid.reshape(-1, self.dy).to(self.dtype).contiguous()
        q, k = int(xq.shape[0]), int(ygrid.shape[0])
        f = out if out is not None else torch.empty((q, k), dtype=torch.float64, device=self.device)
        st = self._lib.cde_density_query(self._h, xq.data_ptr(), q, ygrid.data_ptr(), k,
                                         B.doubles(self._bw(h)), KERNELS[kernel], f.data_ptr(),
                                         _stream_ptr(stream))
        B.check(st, "cde_density_query")
        return f


def launch_batch(items, hx, hy, criterion: str = "cond", stream=None) -> None:
    """One grouped launch (``cde_launch_batch``) of the grid criterion over
    a work list.  ``items``: sequence of (model, i0, i1, totals, nonfinite):
    points [i0, i1) of an FP32 Model, a float64 device tensor [len(hx) *
    len(hy)] that receives the totals when i1 == model.n (else None), and an
    optional int64 device tensor [1] for the non-finite count."""
    hx = [float(v) for v in hx]
    hy = [float(v) for v in hy]
    arr = (B.WorkItem * max(1, len(items)))()
    for k, (m, i0, i1, tot, nonfin) in enumerate(items):
        arr[k].model = m.handle
        arr[k].i0 = int(i0)
        arr[k].i1 = int(i1)
        arr[k].totals_dev = tot.data_ptr() if tot is not None else None
        arr[k].n_nonfinite_dev = nonfin.data_ptr() if nonfin is not None else None
    st = B.load().cde_launch_batch(ctypes.cast(arr, ctypes.c_void_p), len(items), B.doubles(hx), len(hx),
                                   B.doubles(hy), len(hy), CRITERIA[criterion], _stream_ptr(stream))
    B.check(st, "cde_launch_batch")


def density_summary(f: torch.Tensor, ygrid, alpha: float = 0.05, stream=None) -> torch.Tensor:
    """Mass, mode and narrowest 1 - alpha interval of each row of f [q, k]
    on the increasing grid ygrid [k] (``cde_density_summary``): [q, 4] float64."""
    f = f.to(torch.float64).contiguous()
    yg = torch.as_tensor(ygrid, dtype=torch.float64, device=f.device).reshape(-1).contiguous()
    q, k = int(f.shape[0]), int(f.shape[1])
    if yg.numel() != k:
        raise ValueError("ygrid must have one value per column of f")
    out = torch.empty((q, 4), dtype=torch.float64, device=f.device)
    st = B.load().cde_density_summary(f.data_ptr(), yg.data_ptr(), q, k, float(alpha), out.data_ptr(),
                                      _stream_ptr(stream))
    B.check(st, "cde_density_summary")
    return out


def argmax_first_finite(totals) -> int:
    """Index of the first maximum among finite entries (hx-major order)."""
    t = totals.detach().double().cpu()
    finite = torch.isfinite(t)
    if not bool(finite.any()):
        return -1
    t = torch.where(finite, t, torch.full_like(t, -math.inf))
    return int(torch.argmax(t).item())  # torch.argmax returns the first maximal index
