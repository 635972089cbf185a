"""GPU parity of the prefix-sum resamplers (multinomial, Algorithm 7;
systematic, Algorithm 8) through mgp_resample_prefix: every ancestor equals
the oracle's, on ragged sizes around the 2048-weight chunks of the scan, on
weights with zeros and values below the fixed-point resolution, at
N = 2^20 for y = 0..4 and at N = 2^24, y = 4 (the benchmark's size)."""
import numpy as np
import pytest

import oracle
from paper_2109_13504_amd import inputs

pytestmark = pytest.mark.gpu

METHODS = ["multinomial", "systematic"]


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2109_13504_amd import mgp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mgp.lib()
    return torch, torch.device("cuda:0"), mgp


def _mix(n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    w = g.gamma(0.7, 1.0, n).astype(np.float32)
    w[g.integers(0, n, max(1, n // 10))] = 0.0
    w[g.integers(0, n, 3)] = np.float32(1e-30)
    return w


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("n", [1, 2, 33, 1000, 2047, 2048, 2049, 4096, 4097, 100003])
def test_prefix_bit_exact_ragged(env, method, n):
    torch, dev, mgp = env
    r = mgp.PrefixResampler(n)
    for k, w in enumerate([inputs.gaussian_weights(n, 2.0, n % 7), _mix(n, n)]):
        if not (w > 0).any():
            continue
        for seed, sid in ((1, 0), (2**40 + 7, 5)):
            got = r.resample(torch.from_numpy(w).to(dev), method, seed=seed, stream_id=sid).cpu().numpy()
            ref = oracle.resample_prefix(w, method, seed, stream_id=sid)
            np.testing.assert_array_equal(got, ref, err_msg=f"{method} n={n} set={k} seed={seed}")
            st = r.last_stats()
            assert st["status"] == 0 and st["w_max"] == np.float32(w.max())


@pytest.mark.parametrize("y", [0, 1, 2, 3, 4])
def test_prefix_n2pow20(env, y):
    torch, dev, mgp = env
    n = 1 << 20
    w = inputs.gaussian_weights(n, float(y), 0)
    wd = torch.from_numpy(w).to(dev)
    r = mgp.PrefixResampler(n)
    for method in METHODS:
        got = r.resample(wd, method, seed=300 + y).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.resample_prefix(w, method, 300 + y), err_msg=f"{method} y={y}")


def test_prefix_n2pow24_full_array(env):
    torch, dev, mgp = env
    n = 1 << 24
    w = inputs.gaussian_weights(n, 4.0, 0)
    wd = torch.from_numpy(w).to(dev)
    r = mgp.PrefixResampler(n)
    for method in METHODS:
        got = r.resample(wd, method, seed=2024).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.resample_prefix(w, method, 2024), err_msg=method)


@pytest.mark.parametrize("method", METHODS)
def test_prefix_degenerate_weights(env, method):
    torch, dev, mgp = env
    n = 5000
    r = mgp.PrefixResampler(n)
    w = np.zeros(n, np.float32)
    w[4321] = 7.0
    got = r.resample(torch.from_numpy(w).to(dev), method, seed=3).cpu().numpy()
    assert (got == 4321).all()
    for bad in (np.nan, np.inf, -1.0):
        wb = inputs.gaussian_weights(n, 1.0, 2)
        wb[17] = bad
        got = r.resample(torch.from_numpy(wb).to(dev), method, seed=3).cpu().numpy()
        assert (got == -1).all()
        assert r.last_stats()["status"] == mgp.MGP_EWEIGHTS
    got = r.resample(torch.zeros(n, device=dev), method, seed=3).cpu().numpy()
    assert (got == -1).all()


def test_prefix_argument_errors(env):
    torch, dev, mgp = env
    w = torch.ones(100, device=dev)
    r = mgp.PrefixResampler(100)
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_resample_prefix(w.data_ptr(), 100, 2, 1, 0, r.stats.data_ptr(), 0, r.workspace.data_ptr(),
                                r.ws_bytes, 0)
    assert e.value.code == mgp.MGP_EINVAL
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_resample_prefix(w.data_ptr(), 100, 0, 1, 0, r.stats.data_ptr(), 0, r.workspace.data_ptr(), 64, 0)
    assert e.value.code == mgp.MGP_ERANGE
