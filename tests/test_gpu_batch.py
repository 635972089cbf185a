"""Batched mode on the GPU: one plan, one graph launch, many filters of
uneven size. Each filter must equal the oracle and the per-filter launch
path (mgp_batch_run_separate) bit for bit, whatever the launch shape."""
import os

import numpy as np
import pytest

import oracle
from paper_2109_13504_amd import inputs

pytestmark = pytest.mark.gpu

VARIANTS = ["metropolis", "c1", "c2", "megopolis"]


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2109_13504_amd import mgp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mgp.lib()
    return torch, torch.device("cuda:0"), mgp


def make_filters(torch, dev, sizes, ys, d, seeds, with_states=True, Bs=None):
    hosts, fl = [], []
    for f, (n, y) in enumerate(zip(sizes, ys)):
        w, st = inputs.gaussian_weights_and_states(int(n), float(y), max(d, 1), f)
        item = {"w": torch.from_numpy(w).to(dev), "anc": torch.full((int(n),), -7, dtype=torch.int32, device=dev),
                "seed": int(seeds[f]), "stream_id": f, "epsilon": 0.01, "B": int(Bs[f]) if Bs is not None else 0}
        if with_states and d > 0 and f % 3 != 2:  # some filters without a gather
            item["states"] = torch.from_numpy(st).to(dev)
            item["out"] = torch.full((int(n), d), -1.0, dtype=torch.float32, device=dev)
        fl.append(item)
        hosts.append((w, st))
    return fl, hosts


def snapshot(torch, fl):
    torch.cuda.synchronize()
    return [(f["anc"].cpu().numpy().copy(), f["out"].cpu().numpy().copy() if "out" in f else None) for f in fl]


def stats_B(mgp, torch, fl, variant, seeds):
    """B of each filter from the single-filter path (mgp_compute_B)."""
    out = []
    for f, item in enumerate(fl):
        r = mgp.Resampler(item["w"].numel())
        r.compute_B(item["w"], variant, B=item["B"], epsilon=0.01, seed=int(seeds[f]), stream_id=f)
        out.append(r.last_stats()["B"])
    return out


@pytest.mark.parametrize("variant", VARIANTS)
def test_small_ragged_batch_matches_oracle_and_separate(env, variant):
    torch, dev, mgp = env
    sizes = [1, 2, 31, 33, 64, 100, 257, 1000, 1024, 1025, 4097, 5000, 3, 777, 2048, 96]
    ys = np.linspace(0.0, 4.0, len(sizes))
    seeds = [11 + 7 * f for f in range(len(sizes))]
    Bs = [0] * len(sizes)
    Bs[3], Bs[9] = 23, 5  # two explicit B
    d = 3 if variant in ("c1", "metropolis") else 4
    fl, hosts = make_filters(torch, dev, sizes, ys, d, seeds, Bs=Bs)
    plan = mgp.BatchPlan(fl, variant, d=d, block_threads=256, particles_per_thread=4 if variant == "megopolis" else 1,
                         schedule=1)
    plan.run()
    got = snapshot(torch, fl)
    plan.run_separate()
    sep = snapshot(torch, fl)
    Bvals = stats_B(mgp, torch, fl, variant, seeds)
    for f, (w, st) in enumerate(hosts):
        ref = oracle.resample(w, variant, Bvals[f], seeds[f], stream_id=f)
        np.testing.assert_array_equal(got[f][0], ref, err_msg=f"batch {variant} filter {f} n={w.size}")
        np.testing.assert_array_equal(sep[f][0], ref, err_msg=f"separate {variant} filter {f}")
        if got[f][1] is not None:
            np.testing.assert_array_equal(got[f][1], oracle.gather(st, ref))
            np.testing.assert_array_equal(sep[f][1], got[f][1])
    plan.close()


@pytest.mark.parametrize("variant,sched", [("metropolis", 1), ("c1", 1), ("c2", 1), ("c1", 2), ("c2", 2)])
def test_explicit_B_at_every_block_edge(env, variant, sched):
    """One filter per explicit B whose remainder mod 20 puts the chain's
    partial last block at every four-step generator group edge (4, 8, 12,
    16), inside a group (1, 3, 7, 19) and at whole blocks (20, 40), with the
    grid and the persistent schedules."""
    torch, dev, mgp = env
    Bs = [1, 3, 4, 7, 8, 12, 16, 19, 20, 24, 28, 32, 36, 40, 41]
    sizes = [3000 + 37 * f for f in range(len(Bs))]
    ys = np.linspace(0.5, 3.5, len(Bs))
    seeds = [900 + f for f in range(len(Bs))]
    fl, hosts = make_filters(torch, dev, sizes, ys, 2, seeds, Bs=Bs)
    plan = mgp.BatchPlan(fl, variant, d=2, block_threads=256, particles_per_thread=1, schedule=sched)
    plan.run()
    got = snapshot(torch, fl)
    for f, (w, st) in enumerate(hosts):
        ref = oracle.resample(w, variant, Bs[f], seeds[f], stream_id=f)
        np.testing.assert_array_equal(got[f][0], ref, err_msg=f"{variant} B={Bs[f]}")
        if got[f][1] is not None:
            np.testing.assert_array_equal(got[f][1], oracle.gather(st, ref))
    plan.close()


@pytest.mark.parametrize("shape", [(256, 4, 1), (256, 2, 1), (256, 1, 1), (128, 4, 1), (128, 2, 2), (64, 4, 2),
                                   (256, 4, 2)])
def test_megopolis_launch_shapes_agree(env, shape):
    torch, dev, mgp = env
    bt, ppt, sched = shape
    sizes = [1024, 5000, 70000, 33, 12345, 4096]
    ys = [0.5, 4.0, 2.0, 1.0, 3.0, 3.5]
    seeds = [5, 6, 7, 8, 9, 10]
    fl, hosts = make_filters(torch, dev, sizes, ys, 4, seeds)
    plan = mgp.BatchPlan(fl, "megopolis", d=4, block_threads=bt, particles_per_thread=ppt, schedule=sched)
    plan.run()
    got = snapshot(torch, fl)
    Bvals = stats_B(mgp, torch, fl, "megopolis", seeds)
    for f, (w, st) in enumerate(hosts):
        np.testing.assert_array_equal(got[f][0], oracle.resample(w, "megopolis", Bvals[f], seeds[f], stream_id=f))
    plan.close()


@pytest.mark.parametrize("variant,sched", [("metropolis", 2), ("c2", 2), ("c1", 1)])
def test_other_variants_shapes(env, variant, sched):
    torch, dev, mgp = env
    sizes = [3000, 64, 9999]
    seeds = [1, 2, 3]
    fl, hosts = make_filters(torch, dev, sizes, [2.0, 0.0, 4.0], 4, seeds)
    for bt in (64, 128, 256):
        plan = mgp.BatchPlan(fl, variant, d=4, block_threads=bt, particles_per_thread=1, schedule=sched)
        plan.run()
        got = snapshot(torch, fl)
        Bvals = stats_B(mgp, torch, fl, variant, seeds)
        for f, (w, st) in enumerate(hosts):
            np.testing.assert_array_equal(got[f][0], oracle.resample(w, variant, Bvals[f], seeds[f], stream_id=f))
        plan.close()


def test_graph_replays_with_new_seeds(env):
    """Replays of the captured graph, with eager work and synchronisation
    between them, each checked against the per-filter path."""
    torch, dev, mgp = env
    sizes = [2048, 40000, 700, 100000]
    seeds = [1, 2, 3, 4]
    fl, hosts = make_filters(torch, dev, sizes, [1.0, 4.0, 2.0, 3.0], 4, seeds)
    plan = mgp.BatchPlan(fl, "megopolis", d=4, block_threads=256, particles_per_thread=4, schedule=2)
    for rep in range(4):
        new = [1000 * rep + s for s in seeds]
        plan.set_seeds(new)
        plan.run()
        got = snapshot(torch, fl)
        junk = torch.randn(1 << 20, device=dev).sum()  # eager work between replays
        plan.run_separate()
        sep = snapshot(torch, fl)
        for f in range(len(sizes)):
            np.testing.assert_array_equal(got[f][0], sep[f][0], err_msg=f"replay {rep} filter {f}")
            if got[f][1] is not None:
                np.testing.assert_array_equal(got[f][1], sep[f][1])
        del junk
    w0 = hosts[0][0]
    B0 = stats_B(mgp, torch, fl[:1], "megopolis", [3000 + seeds[0]])[0]
    np.testing.assert_array_equal(got[0][0], oracle.resample(w0, "megopolis", B0, 3000 + seeds[0], stream_id=0))
    plan.close()


def test_invalid_filter_is_isolated(env):
    torch, dev, mgp = env
    sizes = [500, 600, 700]
    fl, hosts = make_filters(torch, dev, sizes, [1.0, 1.0, 1.0], 4, [1, 2, 3])
    fl[1]["w"][17] = float("nan")
    plan = mgp.BatchPlan(fl, "megopolis", d=4, block_threads=256, particles_per_thread=4, schedule=1)
    plan.run()
    got = snapshot(torch, fl)
    assert (got[1][0] == -1).all()
    assert np.isnan(got[1][1]).all()
    for f in (0, 2):
        B = stats_B(mgp, torch, fl[f:f + 1], "megopolis", [[1, 2, 3][f]])[0]
        np.testing.assert_array_equal(got[f][0], oracle.resample(hosts[f][0], "megopolis", B, [1, 2, 3][f],
                                                                 stream_id=f))
    plan.close()


def test_autotune_and_cache(env, tmp_path):
    torch, dev, mgp = env
    sizes, ys = inputs.batch_filters(64, 10, 14, seed=5)
    seeds = list(range(64))
    fl, hosts = make_filters(torch, dev, sizes, ys, 4, seeds)
    cache = str(tmp_path / "tune.txt")
    p1 = mgp.BatchPlan(fl, "megopolis", d=4, tune_cache=cache)
    i1 = p1.info()
    assert i1["from_cache"] == 0 and os.path.exists(cache)
    p1.run()
    a = snapshot(torch, fl)
    p2 = mgp.BatchPlan(fl, "megopolis", d=4, tune_cache=cache)
    i2 = p2.info()
    assert i2["from_cache"] == 1
    assert (i2["block_threads"], i2["particles_per_thread"], i2["schedule"]) == \
        (i1["block_threads"], i1["particles_per_thread"], i1["schedule"])
    p2.run()
    b = snapshot(torch, fl)
    for f in range(len(fl)):
        np.testing.assert_array_equal(a[f][0], b[f][0])
    p1.close()
    p2.close()


def test_full_batched_workload(env):
    """512 filters, N_f = round(2^U(10, 18)), y_f ~ U[0, 4], D = 4: the graph
    launch equals the 512 per-filter launch sequences everywhere, and the
    oracle on sampled particles of a subset of filters."""
    torch, dev, mgp = env
    sizes, ys = inputs.batch_filters()
    seeds = [777000 + f for f in range(len(sizes))]
    fl, hosts = make_filters(torch, dev, sizes, ys, 4, seeds)
    plan = mgp.BatchPlan(fl, "megopolis", d=4)
    info = plan.info()
    assert info["filters"] == 512 and info["particles"] == int(np.sum(sizes))
    plan.run()
    got = snapshot(torch, fl)
    plan.run_separate()
    sep = snapshot(torch, fl)
    for f in range(len(fl)):
        np.testing.assert_array_equal(got[f][0], sep[f][0], err_msg=f"filter {f}")
        if got[f][1] is not None:
            np.testing.assert_array_equal(got[f][1], sep[f][1])
    g = np.random.Generator(np.random.PCG64(1))
    for f in g.choice(len(fl), 8, replace=False):
        w, st = hosts[f]
        B = stats_B(mgp, torch, fl[f:f + 1], "megopolis", [seeds[f]])
        # stream_id of this filter is f; stats_B used stream_id 0 for the
        # one-element list, which does not change B
        idx = np.unique(g.integers(0, w.size, 200)).astype(np.int32)
        ref = oracle.resample_subset(w, "megopolis", B[0], seeds[f], idx, stream_id=int(f))
        np.testing.assert_array_equal(got[f][0][idx], ref, err_msg=f"filter {f}")
    plan.close()
