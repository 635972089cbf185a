"""GPU parity: the HIP library (through its C ABI) against the CPU oracle,
bit-exact ancestors and gathered states, on the same seeded inputs.

Sizes: the small single-filter workload (N = 4096, y = 2), ragged sizes that
exercise partial waves, the unrolled-loop tails and the C1/C2 tail partition,
the N = 2^20 sweep over y = 0..4 for all four variants, and N = 2^24 at
y = 4 in the launch configuration the benchmark times (sampled particles,
whose chains the oracle recomputes one by one, and once the full array)."""
import numpy as np
import pytest

import oracle
from paper_2109_13504_amd import inputs

pytestmark = pytest.mark.gpu

VARIANTS = ["metropolis", "c1", "c2", "megopolis"]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def mgp():
    from paper_2109_13504_amd import mgp as m
    m.lib()  # raises if the HIP library is missing
    return m


def _to_dev(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _oracle_B(w, eps=0.01, b_max=65536):
    return oracle.B_from_weights(w, eps, b_max)


def _check_stats(stats, w, eps=0.01):
    st = oracle.reduce(w)
    assert stats["status"] == 0
    assert stats["w_max"] == np.float32(st.w_max)
    assert abs(stats["w_sum"] - st.w_sum) <= 1e-6 * st.w_sum
    B, raw, clamped = oracle.choose_B(st.w_sum, st.w_max, w.size, eps)
    if abs(raw - round(raw)) > 1e-9:
        assert stats["B"] == B, (stats, B, raw)
    assert stats["n"] == w.size


@pytest.mark.parametrize("variant", VARIANTS)
def test_small_config_bit_exact(torch_dev, mgp, variant):
    torch, dev = torch_dev
    n = 4096
    r = mgp.Resampler(n)
    for q in range(3):
        w = inputs.gaussian_weights(n, 2.0, q)
        wd = _to_dev(torch, dev, w)
        for seed in (1, 2**40 + 3):
            anc = r.resample(wd, variant, epsilon=0.01, seed=seed).cpu().numpy()
            stats = r.last_stats()
            _check_stats(stats, w)
            ref = oracle.resample(w, variant, stats["B"], seed)
            np.testing.assert_array_equal(anc, ref, err_msg=f"{variant} q={q} seed={seed}")


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("n", [1, 2, 31, 33, 64, 100, 257, 1000, 4097])
def test_ragged_sizes_and_tails(torch_dev, mgp, variant, n):
    torch, dev = torch_dev
    w = inputs.gaussian_weights(n, 1.0, 3)
    wd = _to_dev(torch, dev, w)
    r = mgp.Resampler(n)
    # B mod 20 covers the partial last block of every size class of the
    # generic chain: inside the first four-step generator group (1, 3), at
    # its edges (4, 8, 12, 16, 24, 36), across the five-step u groups (5, 7),
    # a whole block (20) and the longest remainder (19)
    for B in (1, 3, 4, 5, 7, 8, 12, 16, 19, 20, 23, 24, 36, 41):
        anc = r.resample(wd, variant, B=B, seed=B * 11, stream_id=5).cpu().numpy()
        ref = oracle.resample(w, variant, B, B * 11, stream_id=5)
        np.testing.assert_array_equal(anc, ref, err_msg=f"{variant} n={n} B={B}")


@pytest.mark.parametrize("variant", ["c1", "c2"])
@pytest.mark.parametrize("ps", [4, 8, 128, 1000, 2048, 1 << 20])
def test_partition_sizes(torch_dev, mgp, variant, ps):
    torch, dev = torch_dev
    n = 3000
    w = inputs.gaussian_weights(n, 2.5, 1)
    wd = _to_dev(torch, dev, w)
    anc, stats = mgp.resample(wd, variant, B=27, seed=9, partition_bytes=ps)
    ref = oracle.resample(w, variant, 27, 9, partition_bytes=ps)
    np.testing.assert_array_equal(anc.cpu().numpy(), ref)


@pytest.mark.parametrize("y", [0, 1, 2, 3, 4])
def test_n2pow20_sweep(torch_dev, mgp, y):
    """N = 2^20, y = 0..4, all variants (C1/C2 at 128 and 2048 bytes), with
    the D = 4 gather. Full-array parity for y <= 2, sampled particles above."""
    torch, dev = torch_dev
    n, d = 1 << 20, 4
    w, st = inputs.gaussian_weights_and_states(n, y, d, 0)
    wd, sd = _to_dev(torch, dev, w), _to_dev(torch, dev, st)
    r = mgp.Resampler(n)
    g = np.random.Generator(np.random.PCG64(y))
    sample = np.unique(np.concatenate([np.arange(64), np.arange(n - 64, n), g.integers(0, n, 1500)])).astype(np.int32)
    for variant, ps in [("megopolis", 128), ("metropolis", 128), ("c1", 128), ("c1", 2048), ("c2", 128),
                        ("c2", 2048)]:
        anc_d = r.resample(wd, variant, epsilon=0.01, seed=1000 + y, partition_bytes=ps)
        out = mgp.gather(sd, anc_d)
        anc = anc_d.cpu().numpy()
        stats = r.last_stats()
        _check_stats(stats, w)
        B = stats["B"]
        if y <= 2 and variant in ("megopolis", "metropolis"):
            ref = oracle.resample(w, variant, B, 1000 + y, partition_bytes=ps)
            np.testing.assert_array_equal(anc, ref, err_msg=f"{variant} y={y}")
        else:
            ref = oracle.resample_subset(w, variant, B, 1000 + y, sample, partition_bytes=ps)
            np.testing.assert_array_equal(anc[sample], ref, err_msg=f"{variant}-ps{ps} y={y}")
        assert anc.min() >= 0 and anc.max() < n
        np.testing.assert_array_equal(out.cpu().numpy()[sample], oracle.gather(st, anc[sample]))


def test_n2pow24_sampled(torch_dev, mgp):
    """N = 2^24, y = 4 (B ~ 353), every variant (C1/C2 at 128-byte
    partitions), gather D = 8, in the benchmark's launch configuration."""
    torch, dev = torch_dev
    n, d = 1 << 24, 8
    w, st = inputs.gaussian_weights_and_states(n, 4.0, d, 0)
    wd, sd = _to_dev(torch, dev, w), _to_dev(torch, dev, st)
    r = mgp.Resampler(n)
    g = np.random.Generator(np.random.PCG64(24))
    sample = np.unique(np.concatenate([np.arange(64), np.arange(n - 64, n), g.integers(0, n, 600)])).astype(np.int32)
    for variant in ("megopolis", "metropolis", "c1", "c2"):
        anc_d = r.resample(wd, variant, epsilon=0.01, seed=2024)
        out = mgp.gather(sd, anc_d)
        stats = r.last_stats()
        _check_stats(stats, w)
        anc = anc_d.cpu().numpy()
        ref = oracle.resample_subset(w, variant, stats["B"], 2024, sample)
        np.testing.assert_array_equal(anc[sample], ref, err_msg=variant)
        assert anc.min() >= 0 and anc.max() < n
        np.testing.assert_array_equal(out.cpu().numpy()[sample], st[anc[sample]])
        del out


def test_n2pow24_full_array_megopolis(torch_dev, mgp):
    """Every ancestor and every gathered row at N = 2^24, y = 4, D = 8, in the
    benchmark's launch sequence (mgp_compute_B, then mgp_resample_gather_prepared:
    the accept loop with the fused particle copy), and in the unfused sequence
    (mgp_compute_B, mgp_resample_prepared, mgp_gather). The oracle's chains are
    split over the host's cores (its calls share no state), about 6 x 10^9
    chain steps in all."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    torch, dev = torch_dev
    n, d = 1 << 24, 8
    w, st = inputs.gaussian_weights_and_states(n, 4.0, d, 0)
    wd, sd = _to_dev(torch, dev, w), _to_dev(torch, dev, st)
    r = mgp.Resampler(n)
    r.compute_B(wd, "megopolis", epsilon=0.01, seed=99)
    out_d, anc_d = r.resample_gather_prepared(wd, sd, "megopolis", epsilon=0.01, seed=99)
    out = out_d.cpu().numpy()
    anc = anc_d.cpu().numpy()
    del out_d
    stats = r.last_stats()
    _check_stats(stats, w)
    r.compute_B(wd, "megopolis", epsilon=0.01, seed=99)
    anc_u = r.resample_prepared(wd, "megopolis", epsilon=0.01, seed=99)
    assert torch.equal(anc_u, anc_d)
    out_u = mgp.gather(sd, anc_u).cpu().numpy()
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    parts = np.array_split(np.arange(n, dtype=np.int32), 4 * threads)
    with ThreadPoolExecutor(threads) as ex:
        ref = np.concatenate(list(ex.map(lambda idx: oracle.resample_subset(w, "megopolis", stats["B"], 99, idx),
                                         parts)))
    np.testing.assert_array_equal(anc, ref)
    rows = st[ref]
    np.testing.assert_array_equal(out, rows)
    np.testing.assert_array_equal(out_u, rows)


def test_megopolis_uniform_weights_permutation_at_scale(torch_dev, mgp):
    # a property that holds at any size: with equal weights every candidate
    # is accepted and each offset permutes the particles (32 | N)
    torch, dev = torch_dev
    n = 1 << 22
    wd = torch.full((n,), 0.25, dtype=torch.float32, device=dev)
    anc, _ = mgp.resample(wd, "megopolis", B=9, seed=4)
    assert torch.equal(torch.sort(anc.long()).values, torch.arange(n, device=dev))


@pytest.mark.parametrize("d", [1, 3, 4, 8, 12, 16, 32])
def test_gather_shapes(torch_dev, mgp, d):
    torch, dev = torch_dev
    n_states, n_out = 5000, 7777
    st = inputs.random_states(n_states, d, d)
    anc = np.random.Generator(np.random.PCG64(d)).integers(0, n_states, n_out).astype(np.int32)
    out = mgp.gather(_to_dev(torch, dev, st), _to_dev(torch, dev, anc))
    np.testing.assert_array_equal(out.cpu().numpy(), oracle.gather(st, anc))


def test_gather_out_of_range_ancestor_gives_nan_row(torch_dev, mgp):
    torch, dev = torch_dev
    st = inputs.random_states(10, 4, 1)
    anc = np.array([0, -1, 10, 9], np.int32)
    out = mgp.gather(_to_dev(torch, dev, st), _to_dev(torch, dev, anc)).cpu().numpy()
    np.testing.assert_array_equal(out[0], st[0])
    np.testing.assert_array_equal(out[3], st[9])
    assert np.isnan(out[1]).all() and np.isnan(out[2]).all()


def test_gather_unaligned_rows(torch_dev, mgp):
    torch, dev = torch_dev
    st = inputs.random_states(1001, 4, 2)
    big = _to_dev(torch, dev, np.concatenate([np.zeros(1, np.float32), st.ravel()]))
    view = big[1:].view(1001, 4)  # 4-byte aligned, not 16
    anc = np.arange(1000, -1, -1).astype(np.int32)
    out = mgp.gather(view, _to_dev(torch, dev, anc))
    np.testing.assert_array_equal(out.cpu().numpy(), st[anc])


@pytest.mark.parametrize("bad", [np.nan, np.inf, -1.0])
def test_invalid_weights_poison_ancestors(torch_dev, mgp, bad):
    torch, dev = torch_dev
    w = inputs.gaussian_weights(5000, 1.0)
    w[1234] = bad
    anc, stats = mgp.resample(_to_dev(torch, dev, w), "megopolis", epsilon=0.01)
    assert stats["status"] == mgp.MGP_EWEIGHTS and stats["B"] == 0
    assert (anc.cpu().numpy() == -1).all()


def test_all_zero_weights_rejected(torch_dev, mgp):
    torch, dev = torch_dev
    anc, stats = mgp.resample(torch.zeros(100, device=dev), "metropolis", epsilon=0.01)
    assert stats["status"] == mgp.MGP_EWEIGHTS
    assert (anc.cpu().numpy() == -1).all()


def test_argument_errors(torch_dev, mgp):
    torch, dev = torch_dev
    w = torch.ones(64, device=dev)
    r = mgp.Resampler(64)
    with pytest.raises(mgp.MgpError) as e:
        r.resample(w, "megopolis", B=0, epsilon=0.0)
    assert e.value.code == mgp.MGP_EINVAL
    with pytest.raises(mgp.MgpError) as e:
        r.resample(w, "megopolis", B=70000)
    assert e.value.code == mgp.MGP_ERANGE
    with pytest.raises(mgp.MgpError) as e:
        r.resample(w, "c1", B=3, partition_bytes=6)
    assert e.value.code == mgp.MGP_EINVAL
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_resample(w.data_ptr(), 64, mgp.make_params(B=3), 0, 0, r.workspace.data_ptr(), r.ws_bytes, 0)
    assert e.value.code == mgp.MGP_EINVAL
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_resample(w.data_ptr(), 64, mgp.make_params(B=3), r.stats.data_ptr(), 0, r.workspace.data_ptr(),
                         16, 0)
    assert e.value.code == mgp.MGP_ERANGE


def test_binding_rejects_undersized_or_mistyped_buffers(torch_dev, mgp):
    """The kernels write through plain pointers, so the binding checks every
    caller-supplied buffer before anything is enqueued."""
    torch, dev = torch_dev
    w = torch.ones(64, device=dev)
    r = mgp.Resampler(64)
    sentinel = torch.full((64,), 7, dtype=torch.int32, device=dev)
    for bad in (torch.empty(63, dtype=torch.int32, device=dev), torch.empty(64, dtype=torch.int64, device=dev),
                torch.empty(128, dtype=torch.int32, device=dev)[::2], torch.empty(64, dtype=torch.int32)):
        with pytest.raises(ValueError):
            r.resample(w, "megopolis", B=3, out=bad)
        with pytest.raises(ValueError):
            r.resample_prepared(w, "megopolis", B=3, out=bad)
    with pytest.raises(ValueError):
        r.resample_m(w, 65, "megopolis", B=3, out=sentinel)
    states = torch.zeros((64, 4), device=dev)
    anc = torch.zeros(64, dtype=torch.int32, device=dev)
    with pytest.raises(ValueError):
        mgp.gather(states, anc, out=torch.empty((63, 4), device=dev))
    with pytest.raises(ValueError):
        mgp.BatchPlan([{"w": w, "anc": torch.empty(32, dtype=torch.int32, device=dev), "B": 3}], "megopolis")
    with pytest.raises(ValueError):
        mgp.BatchPlan([{"w": w, "anc": anc, "B": 3, "states": states, "out": torch.empty((64, 2), device=dev)}],
                      "megopolis", d=4)
    torch.cuda.synchronize()
    assert (sentinel == 7).all()


def test_b_clamp_and_explicit_B(torch_dev, mgp):
    torch, dev = torch_dev
    n = 4096
    w = inputs.single_spike_weights(n, 5)
    wd = _to_dev(torch, dev, w)
    r = mgp.Resampler(n, b_max=500)
    anc = r.resample(wd, "megopolis", epsilon=0.01, seed=3).cpu().numpy()
    st = r.last_stats()
    assert st["clamped"] == 1 and st["B"] == 500
    np.testing.assert_array_equal(anc, oracle.resample(w, "megopolis", 500, 3))


def test_results_depend_only_on_seed_and_stream(torch_dev, mgp):
    torch, dev = torch_dev
    n = 20000
    wd = _to_dev(torch, dev, inputs.gaussian_weights(n, 3.0, 2))
    a1, _ = mgp.resample(wd, "megopolis", B=50, seed=1, stream_id=0)
    a2, _ = mgp.resample(wd, "megopolis", B=50, seed=1, stream_id=0)
    a3, _ = mgp.resample(wd, "megopolis", B=50, seed=1, stream_id=1)
    assert torch.equal(a1, a2)
    assert not torch.equal(a1, a3)


def test_split_compute_B_then_prepared_loop(torch_dev, mgp):
    torch, dev = torch_dev
    n = 50000
    w = inputs.gaussian_weights(n, 3.0, 6)
    wd = _to_dev(torch, dev, w)
    r = mgp.Resampler(n)
    for variant in VARIANTS:
        r.compute_B(wd, variant, epsilon=0.01, seed=77, stream_id=3)
        anc = r.resample_prepared(wd, variant, epsilon=0.01, seed=77, stream_id=3).cpu().numpy()
        st = r.last_stats()
        ref = oracle.resample(w, variant, st["B"], 77, stream_id=3)
        np.testing.assert_array_equal(anc, ref, err_msg=variant)
    # a loop whose params do not match the workspace's reduction is refused
    r.compute_B(wd, "megopolis", epsilon=0.01, seed=77, stream_id=3)
    bad = r.resample_prepared(wd, "megopolis", epsilon=0.01, seed=78, stream_id=3).cpu().numpy()
    assert (bad == -1).all()


@pytest.mark.parametrize("n", [1, 31, 257, 4101, 1 << 18, (1 << 18) + 1])
def test_megopolis_small_n_rounds_and_tails(torch_dev, mgp, n):
    """Megopolis up to 2^18 particles runs twenty steps per round of loads;
    B below, at and past multiples of 20 and 5 exercise the rounds and the
    tail. 2^18 + 1 is the first size on the four-particle kernel."""
    torch, dev = torch_dev
    w = inputs.gaussian_weights(n, 2.5, 17)
    wd = _to_dev(torch, dev, w)
    r = mgp.Resampler(n)
    for B in (1, 4, 5, 19, 20, 21, 40, 41, 354):
        got = r.resample(wd, "megopolis", B=B, seed=1000 + B, stream_id=2).cpu().numpy()
        if n <= 4101:
            np.testing.assert_array_equal(got, oracle.resample(w, "megopolis", B, 1000 + B, stream_id=2),
                                          err_msg=f"n={n} B={B}")
        else:
            idx = np.random.Generator(np.random.PCG64(B)).choice(n, 2000, replace=False).astype(np.int32)
            ref = oracle.resample_subset(w, "megopolis", B, 1000 + B, idx, stream_id=2)
            np.testing.assert_array_equal(got[idx], ref, err_msg=f"n={n} B={B}")
