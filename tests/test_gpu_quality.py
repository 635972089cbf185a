"""Resampling quality of the HIP path at N = 2^20 against the paper's own
measurements (Tables 3-6, row 1048576): MSE/N of the offspring counts for
Megopolis, Metropolis, C1 and C2 (128-byte partitions), y = 0..4. The
bit-exact parity tests check sampled particles at this size; this checks
the whole output's statistics."""
import json
import os

import numpy as np
import pytest

from oracle.metrics import QualityAccumulator
from paper_2109_13504_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "mse_over_n_N1048576.json")))
CASES = [(r["variant"], r["partition_bytes"], y, r["mse_over_n"][y]) for r in GOLDEN["rows"] for y in range(5)]


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2109_13504_amd import mgp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mgp.lib()
    return torch, torch.device("cuda:0"), mgp


@pytest.mark.parametrize("variant,ps,y,expect", CASES, ids=[f"{v}-ps{ps}-y{y}" for v, ps, y, _ in CASES])
def test_mse_over_n_at_2pow20(env, variant, ps, y, expect):
    torch, dev, mgp = env
    n = GOLDEN["n"]
    r = mgp.Resampler(n)
    per_run = []
    for q in range(4):
        w = inputs.gaussian_weights(n, y, 40 + q)
        wd = torch.from_numpy(w).to(dev)
        acc = QualityAccumulator(w)
        for k in range(4):
            anc = r.resample(wd, variant, epsilon=GOLDEN["eps"], seed=9000 + 10 * q + k, partition_bytes=ps)
            acc.add(anc.cpu().numpy())
        per_run += [se / n for se in acc.se_list]
    per_run = np.array(per_run)
    est = per_run.mean()
    stderr = per_run.std(ddof=1) / np.sqrt(per_run.size)
    assert abs(est - expect) <= 4 * stderr + 0.01 * expect, (est, expect, stderr)
