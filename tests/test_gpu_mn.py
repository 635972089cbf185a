"""M != N resampling on the GPU (mgp_resample_m) against the oracle, bit for
bit: every variant, m below, equal to and above n, ragged n, B from epsilon
and fixed; m == n equals mgp_resample; the gather of m rows from n states.
Megopolis with m <= n runs the mirrored kernel, m > n the generic one."""
import numpy as np
import pytest

import oracle
from paper_2109_13504_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2109_13504_amd import mgp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mgp.lib()
    return torch, torch.device("cuda:0"), mgp


@pytest.mark.parametrize("variant", ["megopolis", "metropolis", "c1", "c2"])
@pytest.mark.parametrize("n", [5003, 4096])
def test_m_outputs_match_oracle(env, variant, n):
    torch, dev, mgp = env
    w = inputs.gaussian_weights(n, 2.0, 7)
    wd = torch.from_numpy(w).to(dev)
    r = mgp.Resampler(n)
    for m in (1, 777, n - 1, n, n + 1, 3 * n + 17):
        anc = r.resample_m(wd, m, variant, epsilon=0.01, seed=31 + m, stream_id=5, partition_bytes=256)
        torch.cuda.synchronize()
        B = r.last_stats()["B"]
        assert B == oracle.B_from_weights(w, 0.01)[0]
        ref = oracle.resample_m(w, m, variant, B, 31 + m, stream_id=5, partition_bytes=256)
        np.testing.assert_array_equal(anc.cpu().numpy(), ref, err_msg=f"{variant} n={n} m={m}")


@pytest.mark.parametrize("variant", ["megopolis", "metropolis", "c1", "c2"])
def test_m_outputs_fixed_B_at_block_edges(env, variant):
    """Fixed B whose remainder puts the generic chain's partial last block
    inside and at the edges of its generator groups (5-step u groups for
    Megopolis, 4-step j groups of 20-step blocks for the others), m above and
    below n."""
    torch, dev, mgp = env
    n = 3001
    w = inputs.gaussian_weights(n, 1.5, 8)
    wd = torch.from_numpy(w).to(dev)
    r = mgp.Resampler(n)
    for B in (2, 4, 8, 9, 16, 24, 36, 43):
        for m in (2 * n + 5, n - 100):
            anc = r.resample_m(wd, m, variant, B=B, seed=70 + B, stream_id=3)
            ref = oracle.resample_m(w, m, variant, B, 70 + B, stream_id=3)
            np.testing.assert_array_equal(anc.cpu().numpy(), ref, err_msg=f"{variant} B={B} m={m}")


@pytest.mark.parametrize("variant", ["megopolis", "metropolis"])
def test_m_equal_n_is_resample(env, variant):
    torch, dev, mgp = env
    n = 70001
    wd = torch.from_numpy(inputs.gaussian_weights(n, 3.0, 2)).to(dev)
    r = mgp.Resampler(n)
    a = r.resample_m(wd, n, variant, B=40, seed=9).cpu()
    b = r.resample(wd, variant, B=40, seed=9).cpu()
    assert torch.equal(a, b)


def test_large_m_and_gather(env):
    """n = 2^19 inputs, m = 2^21 outputs (generic Megopolis kernel) and
    m = 2^17 (mirrored kernel), then the gather of m rows of d = 4 states."""
    torch, dev, mgp = env
    n = 1 << 19
    w, st = inputs.gaussian_weights_and_states(n, 2.0, 4, 11)
    wd, sd = torch.from_numpy(w).to(dev), torch.from_numpy(st).to(dev)
    r = mgp.Resampler(n)
    for m in (1 << 21, 1 << 17):
        anc = r.resample_m(wd, m, "megopolis", B=16, seed=77)
        out = mgp.gather(sd, anc)
        torch.cuda.synchronize()
        ref = oracle.resample_m(w, m, "megopolis", 16, 77)
        got = anc.cpu().numpy()
        np.testing.assert_array_equal(got, ref)
        np.testing.assert_array_equal(out.cpu().numpy(), oracle.gather(st, ref))


def test_bad_m_rejected(env):
    torch, dev, mgp = env
    wd = torch.ones(100, device=dev)
    r = mgp.Resampler(100)
    with pytest.raises(mgp.MgpError) as e:
        r.resample_m(wd, 0, "megopolis", B=4, out=torch.empty(1, dtype=torch.int32, device=dev))
    assert e.value.code == mgp.MGP_EINVAL
