"""The short paths of mgp_resample: one launch for small filters (n <= 8192
for Megopolis, n <= 4096 for the other variants) and, for Megopolis, two
launches up to 2^15 and the split accept loop up to 2^16. Bit-exact
ancestors against the oracle across sizes on both sides of the limits; for
Megopolis B on both sides of the 20-step passes, 32- and 64-wide segments;
for C1/C2 two partition sizes; stats bit-identical to the three-launch
reduction (mgp_compute_B) for aligned and unaligned weights; invalid
weights; and the workspace left unusable for mgp_resample_prepared."""
import numpy as np
import pytest

import oracle
from paper_2109_13504_amd import inputs

pytestmark = pytest.mark.gpu

SMALL_MAX = 8192


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2109_13504_amd import mgp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mgp.lib()
    return torch, torch.device("cuda:0"), mgp


@pytest.mark.parametrize("n", [1, 2, 31, 32, 100, 4095, 4096, 4101, 6000, SMALL_MAX - 1, SMALL_MAX])
def test_ancestors_match_oracle(env, n):
    torch, dev, mgp = env
    w = inputs.gaussian_weights(n, 3.0, 23)
    wd = torch.from_numpy(w).to(dev)
    r = mgp.Resampler(n)
    for B in (1, 4, 19, 20, 21, 354, 4001):
        if B == 4001 and n > 4101:
            continue  # the oracle's cost; the pass boundary is covered at the smaller sizes
        for seg in (32, 64):
            got = r.resample(wd, "megopolis", B=B, seed=500 + B, stream_id=9, segment=seg).cpu().numpy()
            ref = oracle.resample_m(w, n, "megopolis", B, 500 + B, stream_id=9, segment=seg)
            np.testing.assert_array_equal(got, ref, err_msg=f"n={n} B={B} segment={seg}")
            st = r.last_stats()
            assert st["B"] == B and st["status"] == 0 and st["n"] == n


@pytest.mark.parametrize("variant", ["metropolis", "c1", "c2"])
@pytest.mark.parametrize("n", [1, 2, 31, 100, 4095, 4101, SMALL_MAX])
def test_other_variants_match_oracle(env, variant, n):
    torch, dev, mgp = env
    w = inputs.gaussian_weights(n, 2.5, 41)
    wd = torch.from_numpy(w).to(dev)
    r = mgp.Resampler(n)
    for B in (1, 7, 64):
        for ps in ((128, 512) if variant != "metropolis" else (128,)):
            got = r.resample(wd, variant, B=B, seed=70 + B, stream_id=5, partition_bytes=ps).cpu().numpy()
            ref = oracle.resample(w, variant, B, 70 + B, stream_id=5, partition_bytes=ps)
            np.testing.assert_array_equal(got, ref, err_msg=f"{variant} n={n} B={B} ps={ps}")
    got = r.resample(wd, variant, epsilon=0.01, seed=3).cpu().numpy()
    B = r.last_stats()["B"]
    assert B == oracle.B_from_weights(w, 0.01)[0]
    np.testing.assert_array_equal(got, oracle.resample(w, variant, B, 3))


@pytest.mark.parametrize("n", [SMALL_MAX + 1, 20000, 1 << 15, (1 << 15) + 1, 1 << 16, (1 << 16) + 1])
def test_mid_size_chains(env, n):
    """Past the one-launch limit: up to 2^15 the reduction launch and the split
    accept loop with the finalize step inside; up to 2^16 the three launches
    with the split loop (each particle's draws over four lanes in passes of 20
    steps; B on both sides of the pass boundaries); above, twenty steps'
    loads per round trip."""
    torch, dev, mgp = env
    w = inputs.gaussian_weights(n, 3.0, 77)
    wd = torch.from_numpy(w).to(dev)
    r = mgp.Resampler(n)
    for B in (1, 19, 20, 21, 59, 60, 61, 354):
        got = r.resample(wd, "megopolis", B=B, seed=900 + B, stream_id=6).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.resample(w, "megopolis", B, 900 + B, stream_id=6),
                                      err_msg=f"n={n} B={B}")
    m = n // 2 + 3  # M < N through the same kernels
    got = r.resample_m(wd, m, "megopolis", B=61, seed=5).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.resample_m(w, m, "megopolis", 61, 5))
    # B from epsilon: up to 2^15 the finalize step runs inside the split loop
    # kernel; the stats equal mgp_compute_B's, and the ancestors the oracle's
    got = r.resample(wd, "megopolis", epsilon=0.01, seed=12, stream_id=2).cpu().numpy()
    fused = r.last_stats()
    r.compute_B(wd, "megopolis", epsilon=0.01, seed=12, stream_id=2)
    assert fused == r.last_stats()
    np.testing.assert_array_equal(got, oracle.resample(w, "megopolis", fused["B"], 12, stream_id=2))
    bad = w.copy()
    bad[n // 3] = -1.0
    got = r.resample(torch.from_numpy(bad).to(dev), "megopolis", epsilon=0.01, seed=1).cpu().numpy()
    assert (got == -1).all() and r.last_stats()["status"] == mgp.MGP_EWEIGHTS


def test_two_offset_passes_with_epsilon_and_clamp(env):
    """B from epsilon clamped to b_max = 8003: 400 passes of 20 offsets and
    a tail of 3, in one launch."""
    torch, dev, mgp = env
    n = 2048
    w = inputs.gaussian_weights(n, 4.0, 3)
    w[:] = np.float32(1e-30)
    w[17] = np.float32(1.0)
    wd = torch.from_numpy(w).to(dev)
    r = mgp.Resampler(n, b_max=8003)
    got = r.resample(wd, "megopolis", epsilon=0.01, seed=3).cpu().numpy()
    st = r.last_stats()
    assert st["B"] == 8003 and st["clamped"] == 1
    np.testing.assert_array_equal(got, oracle.resample(w, "megopolis", 8003, 3))


@pytest.mark.parametrize("variant", ["megopolis", "metropolis"])
@pytest.mark.parametrize("n,shift", [(4096, 0), (4096, 1), (4101, 0), (SMALL_MAX, 0), (SMALL_MAX - 3, 1)])
def test_stats_equal_three_launch_reduction(env, variant, n, shift):
    """The fused kernel repeats k_reduce's chunks and thread mapping (float4
    or scalar, by the weights' alignment), so every stats field, the fp64 sum
    included, equals what mgp_compute_B writes for the same weights."""
    torch, dev, mgp = env
    w = inputs.gaussian_weights(n, 2.0, 31)
    base = torch.zeros(n + 4, device=dev)
    wd = base[shift:shift + n]
    wd.copy_(torch.from_numpy(w))
    assert (wd.data_ptr() % 16 == 0) == (shift == 0)
    r = mgp.Resampler(n)
    r.resample(wd, variant, epsilon=0.01, seed=11, stream_id=4)
    fused = r.last_stats()
    r.compute_B(wd, variant, epsilon=0.01, seed=11, stream_id=4)
    three = r.last_stats()
    assert fused == three
    B, _, _ = oracle.B_from_weights(w, 0.01)
    assert fused["B"] == B
    s = oracle.reduce(w).w_sum
    assert abs(fused["w_sum"] - s) <= 1e-12 * s


@pytest.mark.parametrize("variant", ["megopolis", "metropolis", "c1", "c2"])
def test_invalid_weights_and_prepared_refused(env, variant):
    torch, dev, mgp = env
    n = 1000
    w = inputs.gaussian_weights(n, 1.0, 2)
    w[400] = np.nan
    r = mgp.Resampler(n)
    got = r.resample(torch.from_numpy(w).to(dev), variant, epsilon=0.01, seed=1).cpu().numpy()
    assert (got == -1).all() and r.last_stats()["status"] == mgp.MGP_EWEIGHTS
    # a valid call, then a prepared loop with the same params: the one-launch
    # path leaves no offsets or mirror in the workspace, so the loop refuses
    w = inputs.gaussian_weights(n, 1.0, 2)
    wd = torch.from_numpy(w).to(dev)
    r.resample(wd, variant, B=7, seed=1)
    assert (r.resample_prepared(wd, variant, B=7, seed=1).cpu().numpy() == -1).all()


def test_first_size_past_the_limit_uses_three_launches(env):
    torch, dev, mgp = env
    n = SMALL_MAX + 1
    w = inputs.gaussian_weights(n, 3.0, 5)
    wd = torch.from_numpy(w).to(dev)
    r = mgp.Resampler(n)
    got = r.resample(wd, "megopolis", B=41, seed=2).cpu().numpy()
    np.testing.assert_array_equal(got, oracle.resample(w, "megopolis", 41, 2))
    # and the prepared loop works after it, as before
    r.compute_B(wd, "megopolis", B=41, seed=2)
    np.testing.assert_array_equal(r.resample_prepared(wd, "megopolis", B=41, seed=2).cpu().numpy(), got)


@pytest.mark.parametrize("n", [4096, 20000, 50000, 1 << 20])
def test_resample_captured_in_a_graph(env, n):
    """mgp_resample enqueues kernels only (no memset, no allocation), so a
    caller can capture it: the one-, two- and three-launch paths and the
    four-particle loop, replayed with eager work and synchronisation between
    the replays, each replay equal to the oracle."""
    torch, dev, mgp = env
    w = inputs.gaussian_weights(n, 3.0, 88)
    wd = torch.from_numpy(w).to(dev)
    r = mgp.Resampler(n)
    anc = torch.full((n,), -7, dtype=torch.int32, device=dev)
    r.resample(wd, "megopolis", B=40, seed=3, out=anc)  # warm-up outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        r.resample(wd, "megopolis", B=40, seed=3, out=anc)
    idx = np.unique(np.random.Generator(np.random.PCG64(n)).integers(0, n, 3000)).astype(np.int32)
    ref = oracle.resample_subset(w, "megopolis", 40, 3, idx)
    for rep in range(3):
        anc.fill_(-7)
        junk = torch.randn(1 << 18, device=dev).sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(anc.cpu().numpy()[idx], ref, err_msg=f"n={n} replay {rep}")
        del junk
