"""The memory-system probes the benchmark times its ceilings with: they read
what they are asked to read. The streaming probe's per-block sums add up to
passes x the buffer's sum; the pattern probe, over non-negative contents,
leaves its sink untouched (it writes only a negative sum)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2109_13504_amd import mgp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mgp.lib()
    return torch, mgp


@pytest.mark.parametrize("n4,passes,blocks", [(4096, 1, 16), (4096 + 37, 3, 7), (1 << 16, 2, 64)])
def test_stream_read_sums_everything(env, n4, passes, blocks):
    torch, mgp = env
    buf = torch.ones(4 * n4, dtype=torch.float32, device="cuda")
    sink = torch.full((blocks,), -1.0, dtype=torch.float32, device="cuda")
    mgp.mgp_probe_stream_read(buf.data_ptr(), 16 * n4, passes, blocks, sink.data_ptr(),
                              torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert float(sink.double().sum()) == passes * 4 * n4


@pytest.mark.parametrize("n,steps", [(1024, 5), (4096, 20), (1 << 16, 355)])
def test_pattern_read_runs_and_leaves_sink(env, n, steps):
    torch, mgp = env
    mirror = torch.rand(2 * n + 1024, dtype=torch.float32, device="cuda")
    offs = torch.from_numpy(np.random.Generator(np.random.PCG64(n)).integers(0, n + 50, steps)
                            .astype(np.uint32).view(np.int32)).cuda()  # a few past n: clamped
    sink = torch.full((n // 1024,), 7.0, dtype=torch.float32, device="cuda")
    mgp.mgp_probe_pattern_read(mirror.data_ptr(), mirror.numel() * 4, n, offs.data_ptr(), steps, sink.data_ptr(),
                               torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert (sink.cpu().numpy() == 7.0).all()
