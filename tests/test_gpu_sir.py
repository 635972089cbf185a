"""The SIR filter of Section 7 (Algorithm 6) on the GPU against the oracle:
every stage of every step element by element (predicted particles, weights,
ancestors, resampled particles, estimate), whole runs of every variant with
fixed B and with B from epsilon, and of the prefix-sum methods of Table 2's
unbiased rows (multinomial and systematic, Algorithms 7 and 8), the
degenerate step, the graph against the stage-by-stage launches, and launch
shapes. Inputs come from the seeded
generators only; the oracle computes its own chain from them.

Stage 1 evaluates log, cos and exp in fp64 on both sides (device math
library vs. the host C library) and rounds x and w to fp32 once; the fp32
results agree unless an fp64 result falls within an ulp or two of an fp32
rounding boundary (probability about 2^-28 per value), so at these sizes
they are compared bit for bit. The estimate is an fp64 sum of n fp32 values
in a different order on each side: |difference| <= 2 n 2^-53 mean|x|."""
import numpy as np
import pytest

import oracle
from paper_2109_13504_amd import inputs

pytestmark = pytest.mark.gpu

SEED = 0x5EED0000000B


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2109_13504_amd import mgp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mgp.lib()
    return torch, mgp


def problem(R, n, T, traj_seed=inputs.SIR_SEED):
    truth, z = inputs.sir_truth(T, R, seed=traj_seed)
    x0 = np.stack([inputs.sir_initial_particles(n, r) for r in range(R)])
    return truth, z, x0


def mean_tol(x):
    return 2 * x.size * 2.0 ** -53 * float(np.abs(x.astype(np.float64)).mean()) + 1e-300


def make(env, R, n, T, z, x0, **kw):
    torch, mgp = env
    f = mgp.SirFilter(R, n, T, seed=kw.pop("seed", SEED), **kw)
    f.set_measurements(z)
    x0_dev = torch.from_numpy(x0).cuda()
    f.reset(x0_dev)
    torch.cuda.synchronize()
    return f


PREFIX = ("multinomial", "systematic")


def oracle_ancestors(w, variant, B, t, r):
    if variant in PREFIX:
        return oracle.resample_prefix(w, variant, oracle.sir_step_seed(SEED, t), stream_id=r)
    return oracle.resample(w, variant, B, oracle.sir_step_seed(SEED, t), stream_id=r)


@pytest.mark.parametrize("variant", ["megopolis", "metropolis", "c1", "c2", "multinomial", "systematic"])
def test_every_stage_matches_oracle(env, variant):
    torch, mgp = env
    R, n, T, B = 3, 5003, 4, 12
    _, z, x0 = problem(R, n, T)
    f = make(env, R, n, T, z, x0, variant=variant, B=B, use_graph=False)
    xbar = [x0[r].copy() for r in range(R)]
    for t in range(1, T + 1):
        f.predict_update(t)
        gx, gw = f.copy("x").cpu().numpy(), f.copy("w").cpu().numpy()
        f.resample(t)
        ga, gxb = f.copy("ancestors").cpu().numpy(), f.copy("xbar").cpu().numpy()
        f.estimate(t)
        est, bs, st = f.results()
        for r in range(R):
            x, w = oracle.sir_predict_update(xbar[r], t, float(z[r, t]), SEED, r)
            np.testing.assert_array_equal(gx[r], x, err_msg=f"x, step {t} run {r}")
            np.testing.assert_array_equal(gw[r], w, err_msg=f"w, step {t} run {r}")
            anc = oracle_ancestors(w, variant, B, t, r)
            np.testing.assert_array_equal(ga[r], anc, err_msg=f"ancestors, step {t} run {r}")
            xbar[r] = oracle.gather(x, anc).reshape(-1)
            np.testing.assert_array_equal(gxb[r], xbar[r])
            assert abs(est[r, t - 1] - oracle.mean(xbar[r])) <= mean_tol(xbar[r])
            assert bs[r, t - 1] == (1 if variant in PREFIX else B) and st[r, t - 1] == 0
    f.close()


@pytest.mark.parametrize("variant,B", [("megopolis", 16), ("metropolis", 16), ("c1", 16), ("c2", 16),
                                       ("megopolis", 0), ("c2", 0), ("multinomial", 0), ("systematic", 0)])
def test_whole_runs_match_oracle(env, variant, B):
    """T = 30 steps of 4 runs, n ragged; B fixed, or (B = 0) from eq. (bcalc)
    with epsilon = 0.1 at every step as in Section 7."""
    torch, mgp = env
    R, n, T = 4, 4099, 30
    _, z, x0 = problem(R, n, T)
    f = make(env, R, n, T, z, x0, variant=variant, B=B, epsilon=0.1)
    f.run()
    est, bs, st = f.results()
    gxb = f.copy("xbar").cpu().numpy()
    for r in range(R):
        oe, ob, ost, oxb = oracle.sir_filter(x0[r], z[r], variant, B, SEED, r, epsilon=0.1)
        np.testing.assert_array_equal(bs[r], ob, err_msg=f"B, run {r}")
        np.testing.assert_array_equal(st[r], ost)
        np.testing.assert_array_equal(gxb[r], oxb, err_msg=f"last x_bar, run {r}")
        for t in range(T):
            assert abs(est[r, t] - oe[t]) <= 4 * n * 2.0 ** -53 * 40.0, (r, t, est[r, t], oe[t])
    f.close()


def test_graph_equals_stage_by_stage_and_launch_shapes(env):
    torch, mgp = env
    R, n, T = 5, 3000, 12
    _, z, x0 = problem(R, n, T)
    ref = None
    for kw in ({"use_graph": True}, {"use_graph": False}, {"use_graph": True, "block_threads": 128,
                                                           "particles_per_thread": 2},
               {"use_graph": True, "block_threads": 64, "particles_per_thread": 8}):
        f = make(env, R, n, T, z, x0, variant="megopolis", B=20, **kw)
        if kw["use_graph"]:
            f.run()
        else:
            for t in range(1, T + 1):
                f.step(t)
        out = (f.results(), f.copy("xbar").cpu().numpy())
        if ref is None:
            ref = out
        else:
            for a, b in zip(ref[0], out[0]):
                np.testing.assert_array_equal(a, b, err_msg=str(kw))
            np.testing.assert_array_equal(ref[1], out[1])
        # later runs from the same start repeat the first, with eager work
        # and synchronisation between the replays
        for rep in range(3):
            junk = torch.randn(1 << 20, device="cuda").sum()
            f.reset(torch.from_numpy(x0).cuda())
            f.run()
            again = f.results()
            for a, b in zip(again, out[0]):
                np.testing.assert_array_equal(a, b, err_msg=f"{kw} replay {rep}")
            np.testing.assert_array_equal(f.copy("xbar").cpu().numpy(), out[1])
            del junk
        f.close()


@pytest.mark.parametrize("R,n", [(1, 1), (2, 3), (3, 5), (1, 63), (2, 1025), (1, 8192 + 7)])
def test_small_and_ragged_sizes(env, R, n):
    """Sizes that leave partial quads, partial stage-1 blocks and a single
    particle (whose mirror padding repeats it 2048 times)."""
    torch, mgp = env
    T = 6
    _, z, x0 = problem(R, n, T)
    for variant in ("megopolis", "c2", "systematic"):
        f = make(env, R, n, T, z, x0, variant=variant, B=7)
        f.run()
        est, bs, st = f.results()
        gxb = f.copy("xbar").cpu().numpy()
        f.close()
        for r in range(R):
            oe, ob, ost, oxb = oracle.sir_filter(x0[r], z[r], variant, 7, SEED, r)
            np.testing.assert_array_equal(st[r], ost)
            np.testing.assert_array_equal(gxb[r], oxb, err_msg=f"{variant} R={R} n={n} run {r}")
            np.testing.assert_allclose(est[r], oe, rtol=0, atol=4 * n * 2.0 ** -53 * 40.0 + 1e-12)


def test_benchmark_path_100_steps(env):
    """The bench's configuration on a smaller population: Megopolis, B = 16,
    all 100 steps as one graph launch in the default launch shape, 2 runs of
    2^16 particles; every estimate and the final particles against the
    oracle."""
    torch, mgp = env
    R, n, T = 2, 1 << 16, 100
    _, z, x0 = problem(R, n, T)
    f = make(env, R, n, T, z, x0, variant="megopolis", B=16)
    f.run()
    est, bs, st = f.results()
    gxb = f.copy("xbar").cpu().numpy()
    f.close()
    for r in range(R):
        oe, ob, ost, oxb = oracle.sir_filter(x0[r], z[r], "megopolis", 16, SEED, r)
        np.testing.assert_array_equal(st[r], ost)
        np.testing.assert_array_equal(gxb[r], oxb, err_msg=f"run {r}")
        np.testing.assert_allclose(est[r], oe, rtol=0, atol=4 * n * 2.0 ** -53 * 40.0)


@pytest.mark.parametrize("variant", ["megopolis", "multinomial"])
def test_degenerate_step_keeps_predicted_particles(env, variant):
    torch, mgp = env
    R, n, T = 3, 2048, 6
    _, z, x0 = problem(R, n, T)
    z = z.copy()
    z[1, 3] = 1e6  # run 1, step 3: every weight underflows
    f = make(env, R, n, T, z, x0, variant=variant, B=10)
    f.run()
    est, bs, st = f.results()
    assert st[1].tolist() == [0, 0, mgp.MGP_EWEIGHTS, 0, 0, 0] and bs[1, 2] == 0
    assert (st[[0, 2]] == 0).all()
    for r in range(R):
        oe, ob, ost, oxb = oracle.sir_filter(x0[r], z[r], variant, 10, SEED, r)
        np.testing.assert_array_equal(st[r], ost)
        np.testing.assert_array_equal(f.copy("xbar").cpu().numpy()[r], oxb)
        np.testing.assert_allclose(est[r], oe, rtol=0, atol=4 * n * 2.0 ** -53 * 40.0)
    f.close()


def test_stage_order_and_arguments(env):
    torch, mgp = env
    R, n, T = 2, 100, 3
    _, z, x0 = problem(R, n, T)
    f = mgp.SirFilter(R, n, T, variant="megopolis", B=4, seed=1, use_graph=False)
    with pytest.raises(mgp.MgpError) as e:
        f.predict_update(1)  # no reset yet
    assert e.value.code == mgp.MGP_EINVAL
    f.set_measurements(z)
    f.reset(torch.from_numpy(x0).cuda())
    with pytest.raises(mgp.MgpError):
        f.resample(1)  # stage 2 before stage 1
    with pytest.raises(mgp.MgpError) as e:
        f.predict_update(T + 1)
    assert e.value.code == mgp.MGP_ERANGE
    f.step(1)
    with pytest.raises(mgp.MgpError):
        f.run()  # run starts at step 1 only
    f.step(2)
    f.step(3)
    est, _, st = f.results()
    assert np.isfinite(est).all() and (st == 0).all()
    with pytest.raises(ValueError):
        f.reset(torch.zeros(R, n + 1, device="cuda"))
    f.close()
    for bad in ({"runs": 0}, {"n": 0}, {"steps": 0}, {"B": 0, "epsilon": 0.0}, {"variant": 7}):
        kw = dict(runs=2, n=100, steps=3, variant="megopolis", B=4)
        kw.update(bad)
        runs, nn, steps = kw.pop("runs"), kw.pop("n"), kw.pop("steps")
        with pytest.raises(mgp.MgpError):
            mgp.SirFilter(runs, nn, steps, **kw)
