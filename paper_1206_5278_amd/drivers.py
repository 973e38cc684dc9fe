"""Bandwidth-selection drivers on top of the C ABI.

* ``select_grid``: evaluate the exact LOO log-likelihood (eq. 3) on a grid of
  scalar bandwidths and pick the maximiser.  This replaces the random search
  over bandwidths of Section 3.5 by an exhaustive grid.
* ``LooLogLik``: a torch.autograd.Function whose forward is the exact LOO
  log-likelihood S(h) at h = exp(theta) and whose backward is the
  hand-written adjoint (one O(n^2) pass gives value and gradient together).
* ``ascend``: Adam on theta = log h, started at the normal-reference rule
  applied to x and y separately (the baseline of Section 4.2, in its
  textbook form), replacing the random search of Section 3.5.
"""
from __future__ import annotations

import json

import torch

from .model import Model, argmax_first_finite


def select_grid(model: Model, hx, hy, criterion: str = "cond", stream=None):
    """Returns (totals [len(hx), len(hy)] on the host, (a, b) argmax indices)."""
    totals, _, _ = model.loo_grid(hx, hy, criterion, stream=stream)
    t = totals.cpu().reshape(len(hx), len(hy))
    k = argmax_first_finite(t.reshape(-1))
    return t, (k // len(hy), k % len(hy)) if k >= 0 else (-1, -1)


class LooLogLik(torch.autograd.Function):
    """S(exp(theta)) with dS/dtheta = h * dS/dh from the adjoint kernel.

    theta: CPU float64 tensor [dx+dy] (log bandwidths)."""

    @staticmethod
    def forward(ctx, theta, model: Model, criterion: str = "cond"):
        h = torch.exp(theta.detach().double().cpu())
        total, grad, _ = model.loo_grad(h.tolist(), criterion)
        vals = torch.cat([total, grad]).cpu()  # one device round-trip per step
        ctx.save_for_backward(h * vals[1:])
        return vals[0].to(theta.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        (g_theta,) = ctx.saved_tensors
        return grad_out * g_theta.to(grad_out.dtype), None, None


def normal_reference_bandwidths(x, y):
    """h_k = sd_k (4 / ((d + 2) n))^(1/(d+4)) with d = dx + dy, per dimension."""
    x = torch.as_tensor(x, dtype=torch.float64).cpu()
    y = torch.as_tensor(y, dtype=torch.float64).cpu().reshape(x.shape[0], -1)
    n, d = x.shape[0], x.shape[1] + y.shape[1]
    sd = torch.cat([x.std(dim=0), y.std(dim=0)])
    return sd * (4.0 / ((d + 2) * n)) ** (1.0 / (d + 4))


def ascend(model: Model, h0, steps: int = 50, lr: float = 0.05, criterion: str = "cond",
           checkpoint: str | None = None, resume: dict | None = None):
    """Adam (betas 0.9, 0.999) on theta = log h for `steps` steps.

    Returns a dict with the final h, the trace of S per step (S evaluated at
    the parameters before each update) and the Adam state; with `checkpoint`
    the same dict is written as JSON after every step, and `resume` restarts
    from such a dict exactly (evaluations are deterministic)."""
    theta = torch.log(torch.as_tensor(h0, dtype=torch.float64).cpu()).clone().requires_grad_(True)
    opt = torch.optim.Adam([theta], lr=lr, betas=(0.9, 0.999))
    trace, start = [], 0
    if resume is not None:
        with torch.no_grad():
            theta.copy_(torch.tensor(resume["theta"], dtype=torch.float64))
        trace = list(resume["trace"])
        start = int(resume["step"])
        st = opt.state[theta]
        st["step"] = torch.tensor(float(start))
        st["exp_avg"] = torch.tensor(resume["exp_avg"], dtype=torch.float64)
        st["exp_avg_sq"] = torch.tensor(resume["exp_avg_sq"], dtype=torch.float64)
    state = {}
    for step in range(start, steps):
        opt.zero_grad()
        s = LooLogLik.apply(theta, model, criterion)
        (-s).backward()  # maximise S
        trace.append(float(s.detach()))
        opt.step()
        st = opt.state[theta]
        state = {"step": step + 1, "theta": theta.detach().tolist(), "trace": trace,
                 "exp_avg": st["exp_avg"].tolist(), "exp_avg_sq": st["exp_avg_sq"].tolist(),
                 "h": torch.exp(theta.detach()).tolist(), "lr": lr}
        if checkpoint:
            with open(checkpoint, "w") as f:
                json.dump(state, f)
    if not state:
        state = {"step": start, "theta": theta.detach().tolist(), "trace": trace,
                 "h": torch.exp(theta.detach()).tolist(), "lr": lr}
    return state

