"""The headline workload at full size: photoz N = 500,000, dx = 5, dy = 1,
value and bandwidth gradient of the exact LOO log-likelihood (Section 3,
eq. 3 and its derivative) at the normal-reference bandwidths, in the launch
configuration the benchmark times, against the FP64 oracle summed over all
500,000 points.

The oracle's values come from ``tests/golden/photoz500k_headline.json``,
written by ``tests/golden/make_photoz500k_headline.py`` (which calls only the
oracle; about 10 minutes of host CPU).  The test regenerates the seeded FP32
inputs and checks their SHA-256 against the stored one before comparing.
Tolerances: total 1e-6 relative; gradient per component 1e-4 of
max(|g*_k|, 1e-2 max_k |g*_k|); per point 1e-5 max(1, |l*|) on 514 points."""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import workloads
from tests import parity as P

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "photoz500k_headline.json")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_photoz_500k_value_and_gradient_vs_full_oracle():
    print("case: photoz n=500000 value+grad vs the oracle over all points", flush=True)
    import paper_1206_5278_amd as cde
    gold = json.load(open(GOLDEN))
    x, y = workloads.photoz(500_000, seed=0)
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    y32 = np.ascontiguousarray(y, dtype=np.float32)
    digest = hashlib.sha256(x32.tobytes() + y32.tobytes()).hexdigest()
    assert digest == gold["inputs_sha256"], "seeded inputs differ from the ones the oracle ran on"
    m = cde.Model(torch.from_numpy(x32).cuda(), torch.from_numpy(y32).cuda())
    h = gold["h"]
    total, grad, pp = m.loo_grad(h, per_point=True)
    total = float(total.item())
    g = grad.cpu().numpy()
    pp = pp.cpu().numpy()
    ref_total = gold["total"]
    scale = abs(ref_total) if abs(ref_total) >= 0.01 * gold["abs_sum"] else gold["abs_sum"]
    terr = abs(total - ref_total) / scale
    gerr = P.assert_grad(g, np.array(gold["grad"]))
    idx = np.array(gold["sample_idx"])
    perr = P.assert_points(pp[idx], np.array(gold["sample_ell"]))
    print(f"headline: total {total!r} oracle {ref_total!r} rel err {terr:.2e}; "
          f"gradient err {gerr:.2e} of scale; per-point max {perr:.2e}", flush=True)
    assert terr <= P.TOTAL
    m.close()
