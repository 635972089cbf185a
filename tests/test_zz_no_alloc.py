"""mgp_resample_noalloc (the workspace in the library's static scratch)
against mgp_resample (a caller workspace): identical ancestors and stats on
two calls in a row, the second with a smaller input, for every variant; the
largest Megopolis size the scratch holds; and the size limit rejected on the
host before anything is enqueued."""
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


def _both(torch, dev, mgp, w_np, params):
    """(ancestors, stats) of mgp_resample with a caller workspace and of
    mgp_resample_noalloc, on the current stream."""
    n = w_np.size
    w = torch.from_numpy(w_np).to(dev)
    ws_bytes = mgp.mgp_workspace_size(n, params)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    anc_a = torch.empty(n, dtype=torch.int32, device=dev)
    anc_b = torch.full((n,), -7, dtype=torch.int32, device=dev)
    st_a = torch.zeros(mgp.STATS_BYTES, dtype=torch.uint8, device=dev)
    st_b = torch.zeros(mgp.STATS_BYTES, dtype=torch.uint8, device=dev)
    s = mgp.current_stream()
    mgp.mgp_resample(w.data_ptr(), n, params, anc_a.data_ptr(), st_a.data_ptr(), ws.data_ptr(), ws_bytes, s)
    mgp.mgp_resample_noalloc(w.data_ptr(), n, params, anc_b.data_ptr(), st_b.data_ptr(), s)
    torch.cuda.synchronize()
    return anc_a.cpu().numpy(), mgp.decode_stats(st_a), anc_b.cpu().numpy(), mgp.decode_stats(st_b)


@pytest.mark.parametrize("variant", ["megopolis", "metropolis", "c1", "c2"])
def test_noalloc_equals_resample_two_calls(env, variant):
    torch, dev, mgp = env
    # 2^20 runs the reduction, finalize and accept-loop launches; 20000 the
    # two-launch Megopolis path (three launches for the others), which leaves
    # the first call's larger mirror and offsets behind in the scratch
    for n, y, seed in ((1 << 20, 3.0, 21), (20000, 2.0, 22), (3000, 4.0, 23)):
        w_np = inputs.gaussian_weights(n, y, seed)
        p = mgp.make_params(variant, 0, 0.01, 900 + seed, stream_id=5)
        a, sa, b, sb = _both(torch, dev, mgp, w_np, p)
        np.testing.assert_array_equal(b, a, err_msg=f"{variant} n={n}")
        assert sa == sb, (sa, sb)
        assert sb["status"] == 0 and sb["B"] > 1
        idx = np.unique(np.concatenate([np.arange(64), np.arange(n - 64, n), np.arange(0, n, max(1, n // 300))]))
        ref = oracle.resample_subset(w_np, variant, sb["B"], 900 + seed, idx.astype(np.int32), stream_id=5)
        np.testing.assert_array_equal(b[idx], ref, err_msg=f"{variant} n={n} vs oracle")


def test_noalloc_largest_megopolis(env):
    torch, dev, mgp = env
    p = mgp.make_params("megopolis", 0, 0.01, 31)
    # the largest n whose workspace (with the 8n-byte mirror) fits the scratch
    lo, hi = 1, 1 << 24
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if mgp.mgp_workspace_size(mid, p) <= mgp.MGP_NOALLOC_SCRATCH_BYTES:
            lo = mid
        else:
            hi = mid - 1
    n = lo
    assert 8_000_000 < n < 8_400_000
    w_np = inputs.gaussian_weights(n, 1.0, 3)
    a, sa, b, sb = _both(torch, dev, mgp, w_np, p)
    np.testing.assert_array_equal(b, a)
    assert sa == sb
    # one more particle does not fit: rejected before anything is enqueued
    w = torch.ones(n + 1, dtype=torch.float32, device=dev)
    anc = torch.full((n + 1,), -7, dtype=torch.int32, device=dev)
    with pytest.raises(mgp.MgpError) as e:
        mgp.mgp_resample_noalloc(w.data_ptr(), n + 1, p, anc.data_ptr(), 0, mgp.current_stream())
    assert e.value.code == mgp.MGP_ERANGE
    torch.cuda.synchronize()
    assert (anc.cpu().numpy() == -7).all()
