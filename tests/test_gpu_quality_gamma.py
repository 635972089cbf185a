"""Resampling quality on gamma-distributed weights (eq. (gammaEq), rate 1,
shape 0.5, 2, 3, 10, 50; the paper's appendix shows this study as a figure
only, so its values are parity unpinned). N = 2^20, eps = 0.01.

What is checked:
  - Metropolis: with B from eq. (proposition) each output's ancestor follows
    the normalised weights up to the bias bound, so the offspring counts are
    close to multinomial and MSE/N = 1 - sum p_i^2 (about 1 here);
  - the orderings the paper states for these weights: Megopolis has the
    lowest MSE of Megopolis, Metropolis, C1 and C2 (128-byte partitions), and
    C1-PS128 is worse than Megopolis.
The values are printed (pytest -s) for the design record."""
import numpy as np
import pytest

from oracle.metrics import QualityAccumulator
from paper_2109_13504_amd import inputs

pytestmark = pytest.mark.gpu

ALPHAS = [0.5, 2.0, 3.0, 10.0, 50.0]
VARIANTS = ["megopolis", "metropolis", "c1", "c2"]


@pytest.fixture(scope="module")
def mse():
    import torch

    from paper_2109_13504_amd import mgp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dev = torch.device("cuda:0")
    n = 1 << 20
    r = mgp.Resampler(n)
    table = {}
    for a in ALPHAS:
        seqs = [inputs.gamma_weights(n, a, q) for q in range(2)]
        for v in VARIANTS:
            per = []
            for q, w in enumerate(seqs):
                wd = torch.from_numpy(w).to(dev)
                acc = QualityAccumulator(w)
                for k in range(4):
                    anc = r.resample(wd, v, epsilon=0.01, seed=500 + 10 * q + k, partition_bytes=128)
                    acc.add(anc.cpu().numpy())
                per += [se / n for se in acc.se_list]
            per = np.array(per)
            table[(a, v)] = (per.mean(), per.std(ddof=1) / np.sqrt(per.size), r.last_stats()["B"])
    for a in ALPHAS:
        print(f"gamma alpha={a:g}: " + ", ".join(f"{v} {table[(a, v)][0]:.4f} (B={table[(a, v)][2]})"
                                                 for v in VARIANTS))
    return table


@pytest.mark.parametrize("alpha", ALPHAS)
def test_metropolis_is_near_multinomial(mse, alpha):
    w = inputs.gamma_weights(1 << 20, alpha, 0).astype(np.float64)
    p = w / w.sum()
    expect = 1.0 - float(np.sum(p * p))
    est, se, _ = mse[(alpha, "metropolis")]
    assert abs(est - expect) <= 4 * se + 0.01, (est, expect, se)


@pytest.mark.parametrize("alpha", ALPHAS)
def test_megopolis_lowest_mse(mse, alpha):
    mego = mse[(alpha, "megopolis")][0]
    for v in ("metropolis", "c1", "c2"):
        assert mego < mse[(alpha, v)][0], (alpha, v, mego, mse[(alpha, v)][0])
    assert mse[(alpha, "c1")][0] > mego
