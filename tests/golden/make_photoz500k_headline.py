"""Writes ``photoz500k_headline.json``: the FP64 oracle's value and gradient of
the exact leave-one-out log-likelihood (Section 3, eq. 3, conditional form of
the A_i expansion of Section 3.2, and its derivative with respect to the
diagonal bandwidths) on the photoz-shaped workload at N = 500,000, dx = 5,
dy = 1, summed over ALL 500,000 points.

Only ``oracle/`` computes: the data are the seeded draws of ``workloads``
rounded once to FP32 (the arrays an FP32 run receives), promoted exactly to
FP64.  The bandwidths are the normal-reference rule applied per dimension,
h_k = sd_k (4 / ((d + 2) n))^(1/(d + 4)) with d = dx + dy and the sample
standard deviation (n - 1 denominator); they are stored, and the test uses
the stored values.

Stored: a SHA-256 of the FP32 input bytes (the test checks its own inputs
against it), h, the total S* (index-order compensated sum), sum_i |l*_i|
(the total tolerance's scale when S* is a cancellation), the gradient
dS*/dh (each component an index-order compensated sum), and l*_i for 512
seeded sample points plus the points of smallest and largest l*_i.

Run: ``python -m tests.golden.make_photoz500k_headline [--threads T]``
(about 10 minutes on 8 threads).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "photoz500k_headline.json")
N = 500_000


def inputs():
    """The FP32 arrays of the headline workload and their SHA-256."""
    import workloads
    x, y = workloads.photoz(N, seed=0)
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    y32 = np.ascontiguousarray(y, dtype=np.float32)
    digest = hashlib.sha256(x32.tobytes() + y32.tobytes()).hexdigest()
    return x32, y32, digest


def main():
    import oracle
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    x32, y32, digest = inputs()
    xo, yo = x32.astype(np.float64), y32.astype(np.float64)
    d = xo.shape[1] + yo.shape[1]
    sd = np.concatenate([xo.std(axis=0, ddof=1), yo.std(axis=0, ddof=1)])
    h = sd * (4.0 / ((d + 2) * N)) ** (1.0 / (d + 4))
    ells, dells = [], []
    t0 = time.perf_counter()
    for c in range(10):
        idx = np.arange(c * N // 10, (c + 1) * N // 10)
        ell, dell = oracle.loo(xo, yo, h, idx=idx, grad=True, nthreads=args.threads)
        ells.append(ell)
        dells.append(dell)
        print(f"slice {c + 1}/10 ({time.perf_counter() - t0:.0f} s)", flush=True)
    ell = np.concatenate(ells)
    dell = np.concatenate(dells)
    rng = np.random.default_rng(2024)
    sample = np.sort(rng.choice(N, 512, replace=False))
    sample = np.unique(np.concatenate([sample, [int(np.argmin(ell)), int(np.argmax(ell))]]))
    out = {
        "workload": "photoz N=500000 dx=5 dy=1 seed 0, FP32 inputs; normal-reference diagonal h; "
                    "conditional criterion",
        "inputs_sha256": digest,
        "h": h.tolist(),
        "total": oracle.total(ell),
        "abs_sum": oracle.total(np.abs(ell)),
        "grad": [oracle.total(dell[:, k]) for k in range(d)],
        "sample_idx": sample.tolist(),
        "sample_ell": ell[sample].tolist(),
        "oracle_threads": args.threads,
        "oracle_seconds": round(time.perf_counter() - t0, 1),
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"wrote {OUT}: total {out['total']!r}")


if __name__ == "__main__":
    main()
