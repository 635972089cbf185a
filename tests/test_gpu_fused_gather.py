"""GPU parity of the fused entry points mgp_resample_gather and
mgp_resample_gather_prepared: the accept loop copies x_bar_i = x_{k_i} (the
last statement of Algorithms 2-5) while the ancestor is in a register.

Each case checks ancestors and rows against the oracle (every particle at
small sizes, first/last 64 plus random ones above) and against the unfused
mgp_resample + mgp_gather on the same arguments, bit for bit. Sizes cover
every launch path of mgp_resample (one launch up to 8192 / 4096 particles,
two up to 32768 for Megopolis, the split, deep and four-particle loops
beyond) and every row-copy form (float4 rows of 1, 2 and 4 vectors compiled
in, other float4 widths, scalar rows, unaligned rows)."""
import numpy as np
import pytest

import oracle
from paper_2109_13504_amd import inputs

pytestmark = pytest.mark.gpu

VARIANTS = ["megopolis", "metropolis", "c1", "c2"]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def mgp():
    from paper_2109_13504_amd import mgp as m
    m.lib()
    return m


def _dev(torch, dev, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _sample(n, seed, k=600):
    g = np.random.Generator(np.random.PCG64(seed))
    idx = np.concatenate([np.arange(min(n, 64)), np.arange(max(0, n - 64), n), g.integers(0, n, k)])
    return np.unique(idx).astype(np.int32)


def _fused_vs_unfused_and_oracle(torch, dev, mgp, n, d, variant, y=2.5, B=0, seed=5, stream_id=0, full=False):
    w, st = inputs.gaussian_weights_and_states(n, y, d, 3)
    wd, sd = _dev(torch, dev, w), _dev(torch, dev, st)
    r = mgp.Resampler(n)
    eps = 0.01
    out, anc = r.resample_gather(wd, sd, variant, B=B, epsilon=eps, seed=seed, stream_id=stream_id)
    stats = r.last_stats()
    assert stats["status"] == 0
    Bu = stats["B"]
    anc_u = r.resample(wd, variant, B=B, epsilon=eps, seed=seed, stream_id=stream_id)
    out_u = mgp.gather(sd, anc_u)
    assert torch.equal(anc, anc_u), f"{variant} n={n}: fused ancestors differ from mgp_resample"
    assert torch.equal(out, out_u), f"{variant} n={n} d={d}: fused rows differ from mgp_gather"
    a = anc.cpu().numpy()
    o = out.cpu().numpy()
    if full:
        ref = oracle.resample(w, variant, Bu, seed, stream_id=stream_id)
        np.testing.assert_array_equal(a, ref, err_msg=f"{variant} n={n}")
        np.testing.assert_array_equal(o, oracle.gather(st, ref))
    else:
        idx = _sample(n, n + d)
        ref = oracle.resample_subset(w, variant, Bu, seed, idx, stream_id=stream_id)
        np.testing.assert_array_equal(a[idx], ref, err_msg=f"{variant} n={n}")
        np.testing.assert_array_equal(o[idx], oracle.gather(st, ref))
        np.testing.assert_array_equal(o, st[a])
    return Bu


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("n,d", [(4096, 4), (4096, 8), (1000, 3), (33, 16), (1, 8)])
def test_fused_one_launch_sizes_full_oracle(torch_dev, mgp, variant, n, d):
    """The one-launch path (n <= 8192 Megopolis, <= 4096 the others), every
    particle and row against the oracle."""
    torch, dev = torch_dev
    _fused_vs_unfused_and_oracle(torch, dev, mgp, n, d, variant, full=True)


@pytest.mark.parametrize("n", [8193, 20000, 32768, 50000, (1 << 17) + 3, (1 << 18) + 1, 300001])
@pytest.mark.parametrize("d", [4, 8, 16, 12, 5])
def test_fused_megopolis_every_launch_path(torch_dev, mgp, n, d):
    """Megopolis past one launch: two launches with the finalize step in the
    split loop (<= 32768), the split loop (<= 2^16), the deep loop (<= 2^18),
    the four-particle loop beyond; rows of 1, 2, 4 float4s (compiled in), 3
    float4s and 5 floats."""
    torch, dev = torch_dev
    _fused_vs_unfused_and_oracle(torch, dev, mgp, n, d, "megopolis", y=3.0)


@pytest.mark.parametrize("variant", ["metropolis", "c1", "c2"])
@pytest.mark.parametrize("n", [4097, 70001])
def test_fused_baselines_generic_loop(torch_dev, mgp, variant, n):
    torch, dev = torch_dev
    _fused_vs_unfused_and_oracle(torch, dev, mgp, n, 8, variant, y=3.0)


@pytest.mark.parametrize("y", [0, 2, 4])
def test_fused_n2pow20_d4_all_variants(torch_dev, mgp, y):
    """N = 2^20 with the D = 4 gather: the four variants, sampled chains and
    every row."""
    torch, dev = torch_dev
    for variant in VARIANTS:
        _fused_vs_unfused_and_oracle(torch, dev, mgp, 1 << 20, 4, variant, y=float(y), seed=1000 + y)


def test_fused_prepared_and_explicit_B_tails(torch_dev, mgp):
    """mgp_compute_B + mgp_resample_gather_prepared with explicit B across the
    five-step block tails, stream_id != 0, on the four-particle loop."""
    torch, dev = torch_dev
    n, d = (1 << 18) + 1024, 8
    w, st = inputs.gaussian_weights_and_states(n, 2.0, d, 7)
    wd, sd = _dev(torch, dev, w), _dev(torch, dev, st)
    r = mgp.Resampler(n)
    idx = _sample(n, 9)
    for B in (1, 4, 5, 6, 23, 354):
        r.compute_B(wd, "megopolis", B=B, seed=B, stream_id=6)
        out, anc = r.resample_gather_prepared(wd, sd, "megopolis", B=B, seed=B, stream_id=6)
        a = anc.cpu().numpy()
        ref = oracle.resample_subset(w, "megopolis", B, B, idx, stream_id=6)
        np.testing.assert_array_equal(a[idx], ref, err_msg=f"B={B}")
        np.testing.assert_array_equal(out.cpu().numpy(), st[a])


def test_fused_without_ancestor_array(torch_dev, mgp):
    """ancestors_dev = NULL: the rows alone, equal to the run that writes
    ancestors, on each Megopolis path."""
    torch, dev = torch_dev
    for n in (4096, 20000, 1 << 17, 1 << 19):
        w, st = inputs.gaussian_weights_and_states(n, 3.0, 8, 1)
        wd, sd = _dev(torch, dev, w), _dev(torch, dev, st)
        r = mgp.Resampler(n)
        out_a, anc = r.resample_gather(wd, sd, "megopolis", epsilon=0.01, seed=3)
        out_b, none = r.resample_gather(wd, sd, "megopolis", epsilon=0.01, seed=3, with_anc=False)
        assert none is None
        assert torch.equal(out_a, out_b), n


def test_fused_unaligned_rows(torch_dev, mgp):
    """States 4-byte but not 16-byte aligned: the scalar row copy."""
    torch, dev = torch_dev
    n = 300001
    w, st = inputs.gaussian_weights_and_states(n, 2.0, 4, 2)
    big = _dev(torch, dev, np.concatenate([np.zeros(1, np.float32), st.ravel()]))
    view = big[1:].view(n, 4)
    r = mgp.Resampler(n)
    out, anc = r.resample_gather(_dev(torch, dev, w), view, "megopolis", epsilon=0.01, seed=8)
    a = anc.cpu().numpy()
    np.testing.assert_array_equal(out.cpu().numpy(), st[a])
    idx = _sample(n, 4)
    np.testing.assert_array_equal(a[idx], oracle.resample_subset(w, "megopolis", r.last_stats()["B"], 8, idx))


@pytest.mark.parametrize("n", [4096, 20000, 1 << 17, (1 << 18) + 1])
@pytest.mark.parametrize("variant", ["megopolis", "c2"])
def test_fused_invalid_weights_give_nan_rows(torch_dev, mgp, n, variant):
    torch, dev = torch_dev
    w, st = inputs.gaussian_weights_and_states(n, 1.0, 4, 0)
    w[n // 3] = np.nan
    r = mgp.Resampler(n)
    out, anc = r.resample_gather(_dev(torch, dev, w), _dev(torch, dev, st), variant, epsilon=0.01, seed=1)
    assert r.last_stats()["status"] == mgp.MGP_EWEIGHTS
    assert (anc.cpu().numpy() == -1).all()
    assert np.isnan(out.cpu().numpy()).all()


def test_fused_argument_errors(torch_dev, mgp):
    torch, dev = torch_dev
    n = 64
    w = torch.ones(n, device=dev)
    st = torch.zeros((n, 4), device=dev)
    r = mgp.Resampler(n)
    p = mgp.make_params(B=3)
    with pytest.raises(mgp.MgpError) as e:  # out overlaps states
        mgp.mgp_resample_gather(w.data_ptr(), n, p, st.data_ptr(), 4, 0, st.data_ptr() + 16, 0,
                                r.workspace.data_ptr(), r.ws_bytes, 0)
    assert e.value.code == mgp.MGP_EINVAL
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_resample_gather(w.data_ptr(), n, p, st.data_ptr(), 0, 0, st.data_ptr(), 0,
                                r.workspace.data_ptr(), r.ws_bytes, 0)
    assert e.value.code == mgp.MGP_EINVAL
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_resample_gather_prepared(w.data_ptr(), n, p, 0, 4, 0, st.data_ptr(), r.workspace.data_ptr(),
                                         r.ws_bytes, 0)
    assert e.value.code == mgp.MGP_EINVAL
    with pytest.raises(ValueError):
        r.resample_gather(w, torch.zeros((n - 1, 4), device=dev), "megopolis", B=3)
