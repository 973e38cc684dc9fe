"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module holds random-number draws only: none of the estimator's
arithmetic lives here, so that the oracle (``oracle/``) and the HIP library
(``paper_1206_5278_amd``) can both consume the same arrays without sharing
any code that computes the method.

The paper's own datasets (geyser, SDSS DR4 positions, census, SDSS redshift;
Section 4) are not available; each generator below is a stand-in with the
shape, dimensionality and value structure of one benchmark workload:

* ``tiny``      -- N=2000, dx=dy=1, the bimodal-then-unimodal conditional
                   density of Figure 1 (FP64 workload).
* ``gmm``       -- N=50k, dx=5, dy=1, a 10-component 6-D Gaussian mixture.
* ``photoz``    -- N=500k, dx=5, dy=1, photometric-redshift-shaped data
                   (the role of the SDSS redshift study, Section 4.3).
* ``highdim``   -- N=1M, dx=16, dy=2, a 20-component 16-D mixture with
                   y = tanh(W x) + noise.
* ``serve_stream`` -- the Poisson request stream for the serving workload.

Conventions: N(mu, s) with a scalar s means standard deviation s; N(0, S)
with a matrix S means covariance S; Gamma(k, theta) is shape/scale.
All generators use numpy's PCG64 (``numpy.random.default_rng``) and return
float64 arrays; ``as_f32`` rounds once to float32 (the array that an FP32
run -- and the oracle checking it -- both read).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "tiny", "gmm", "photoz", "highdim", "gmm_general", "as_f32", "geomspace",
    "subsample", "Request", "serve_stream", "WORKLOADS",
]


def geomspace(lo: float, hi: float, g: int) -> np.ndarray:
    """g log-spaced values from lo to hi inclusive, in float64."""
    return np.geomspace(lo, hi, g)


def as_f32(a: np.ndarray) -> np.ndarray:
    """Round a float64 array once to float32 (C-contiguous)."""
    return np.ascontiguousarray(a, dtype=np.float32)


def tiny(n: int = 2000, seed: int = 0):
    """x ~ U(0,100); for x < 50, y is an equal mixture of N(20+0.3x, 5) and
    N(80-0.3x, 5); otherwise y ~ N(50, 8)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 100.0, size=n)
    comp = rng.integers(0, 2, size=n)
    lo_mean = np.where(comp == 0, 20.0 + 0.3 * x, 80.0 - 0.3 * x)
    y_lo = rng.normal(lo_mean, 5.0)
    y_hi = rng.normal(50.0, 8.0, size=n)
    y = np.where(x < 50.0, y_lo, y_hi)
    return x.reshape(n, 1), y.reshape(n, 1)


def gmm_general(n: int, d: int, seed: int, k: int = 10, lo: float = -5.0,
                hi: float = 5.0):
    """n draws of a k-component d-D Gaussian mixture: means U(lo,hi)^d,
    covariances A A^T / d + 0.1 I with A ~ N(0,1) (d x d), equal weights."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(lo, hi, size=(k, d))
    chol = []
    for _ in range(k):
        a = rng.normal(0.0, 1.0, size=(d, d))
        cov = a @ a.T / d + 0.1 * np.eye(d)
        chol.append(np.linalg.cholesky(cov))
    comp = rng.integers(0, k, size=n)
    z = rng.normal(0.0, 1.0, size=(n, d))
    out = np.empty((n, d))
    for c in range(k):
        sel = comp == c
        out[sel] = means[c] + z[sel] @ chol[c].T
    return out


def gmm(n: int = 50_000, seed: int = 0, dx: int = 5):
    """(x, y) jointly from a 10-component (dx+1)-D mixture; x is the first
    dx coordinates and y the last."""
    v = gmm_general(n, dx + 1, seed)
    return np.ascontiguousarray(v[:, :dx]), np.ascontiguousarray(v[:, dx:])


def photoz(n: int = 500_000, seed: int = 0):
    """z ~ Gamma(shape 2, scale 0.08) clipped to [0, 0.6]; five features
    x_k = z c_k + 0.1 t_4 with c_k ~ U(1,4) drawn once per feature;
    y = z + N(0, 0.02)."""
    rng = np.random.default_rng(seed)
    z = np.clip(rng.gamma(2.0, 0.08, size=n), 0.0, 0.6)
    c = rng.uniform(1.0, 4.0, size=5)
    x = z[:, None] * c[None, :] + 0.1 * rng.standard_t(4.0, size=(n, 5))
    y = z + rng.normal(0.0, 0.02, size=n)
    return x, y.reshape(n, 1)


def highdim(n: int = 1_000_000, seed: int = 0):
    """x from a 20-component isotropic 16-D mixture (means U(-3,3)^16,
    per-component sd U(0.5,1.5)); y = tanh(W x) + N(0, 0.1 I_2) with W
    entries N(0, 1/16) (sd 0.25), W of shape 2 x 16."""
    rng = np.random.default_rng(seed)
    k, d = 20, 16
    means = rng.uniform(-3.0, 3.0, size=(k, d))
    sds = rng.uniform(0.5, 1.5, size=k)
    w = rng.normal(0.0, 0.25, size=(2, d))
    comp = rng.integers(0, k, size=n)
    x = means[comp] + sds[comp, None] * rng.normal(0.0, 1.0, size=(n, d))
    y = np.tanh(x @ w.T) + rng.normal(0.0, math.sqrt(0.1), size=(n, 2))
    return x, y


def subsample(x: np.ndarray, y: np.ndarray, m: int, seed: int = 1):
    """A seeded subset of m rows (without replacement), kept in index order."""
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(x.shape[0], size=m, replace=False))
    return np.ascontiguousarray(x[idx]), np.ascontiguousarray(y[idx])


@dataclasses.dataclass
class Request:
    """One request of the serving stream.

    kind 'job': bandwidth selection over a 16 x 16 grid on its own data
    (n points, dx features, dy=1).  kind 'query': q query points evaluated
    on a 256-point y grid against resident training set ``set_id``."""
    rid: int
    t_arrive: float
    kind: str
    n: int = 0
    dx: int = 0
    seed: int = 0
    set_id: int = -1
    q: int = 0


def serve_stream(rate: float = 200.0, duration: float = 60.0, seed: int = 0,
                 p_query: float = 0.7, n_lo: int = 1000, n_hi: int = 200_000,
                 q_max: int = 4096, n_sets: int = 8):
    """Open-loop Poisson arrivals; 70% queries (q ~ U{1..q_max}), 30% jobs
    (n log-uniform in [n_lo, n_hi], dx ~ U{1..8}, dy = 1)."""
    rng = np.random.default_rng(seed)
    t, rid, out = 0.0, 0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        if rng.uniform() < p_query:
            out.append(Request(rid, t, "query", set_id=int(rng.integers(0, n_sets)),
                               q=int(rng.integers(1, q_max + 1))))
        else:
            n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
            out.append(Request(rid, t, "job", n=n, dx=int(rng.integers(1, 9)),
                               seed=int(rng.integers(0, 2**31 - 1))))
        rid += 1
    return out


def resident_sets(n_sets: int = 8, seed: int = 0, n_lo: int = 1000,
                  n_hi: int = 200_000):
    """The serving workload's resident training sets, drawn like the jobs."""
    rng = np.random.default_rng(seed + 7919)
    sets = []
    for s in range(n_sets):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        dx = int(rng.integers(1, 9))
        x, y = gmm(n, seed=int(rng.integers(0, 2**31 - 1)), dx=dx)
        sets.append((x, y))
    return sets


WORKLOADS = {
    "tiny": dict(n=2000, dx=1, dy=1, grid=(geomspace(0.5, 20.0, 8), geomspace(0.5, 20.0, 8)),
                 precision="f64"),
    "gmm": dict(n=50_000, dx=5, dy=1, grid=(geomspace(0.05, 5.0, 32), geomspace(0.05, 5.0, 32)),
                precision="f32"),
    # scalar grid on the same data: 1/4x to 4x the normal-reference scale
    # (hx about 0.08, hy about 0.028 at n = 500,000)
    "photoz": dict(n=500_000, dx=5, dy=1, precision="f32", steps=50,
                   grid=(geomspace(0.02, 0.32, 16), geomspace(0.007, 0.112, 16))),
    "highdim": dict(n=1_000_000, dx=16, dy=2,
                    grid=(geomspace(0.2, 5.0, 16), geomspace(0.02, 1.0, 16)), precision="f32"),
}
