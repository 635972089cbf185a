"""The index paths for very large N, at real sizes: Megopolis above the
mirror limit (2^29 - 4096 particles, where the per-load wrap of Algorithm 5
is used) and every variant above 2^30 particles (64-bit weight indexing).
Weights are uniform (0, 1] draws made on the device; the oracle recomputes
sampled particles' chains from the same fp32 bytes."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2109_13504_amd import mgp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mgp.lib()
    return torch, torch.device("cuda:0"), mgp


def _check(torch, dev, mgp, n, variants, B=9):
    g = torch.Generator(device=dev)
    g.manual_seed(n % 1000003)
    w = torch.rand(n, generator=g, device=dev, dtype=torch.float32) + 1e-6
    w_np = w.cpu().numpy()
    r = mgp.Resampler(n)
    rng = np.random.Generator(np.random.PCG64(n % 7919))
    sample = np.unique(np.concatenate([np.arange(70), np.arange(n - 70, n),
                                       rng.integers(0, n, 300)])).astype(np.int32)
    for variant in variants:
        anc = r.resample(w, variant, B=B, seed=31, stream_id=2)
        got = anc[torch.from_numpy(sample).to(dev).long()].cpu().numpy()
        ref = oracle.resample_subset(w_np, variant, B, 31, sample, stream_id=2)
        np.testing.assert_array_equal(got, ref, err_msg=f"{variant} n={n}")
        assert int(anc.min()) >= 0 and int(anc.max()) < n
        del anc
    del w, r


def test_megopolis_past_the_mirror_limit(env):
    torch, dev, mgp = env
    _check(torch, dev, mgp, (1 << 29) + 96, ["megopolis"])


def test_wide_indexing_above_2pow30(env):
    torch, dev, mgp = env
    _check(torch, dev, mgp, (1 << 30) + 37, ["megopolis", "metropolis", "c2"], B=7)
