"""The SIR experiment of Section 7 at the paper's particle count against
Table 2 (tests/golden/sir_table2.json): 16 ground-truth trajectories, 2^20
particles, 100 steps, fewer Monte Carlo runs than the paper's 50 (4 per
trajectory). The trajectories are this repository's synthetic ones, not the
paper's, so the RMSE is held to a band around the printed value; the
orderings Table 2 shows are checked on the same trajectories for all twelve
resampler rows (four variants x B = 16, 32, 64): C1 with 128-byte partitions
is the worst at every B, the other three are close, and every variant
improves with B; so are the claims of the B study."""
import json
import os

import numpy as np
import pytest

from paper_2109_13504_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sir_table2.json")))
PAPER = {(r["variant"], r["B"]): r["rmse"] for r in GOLDEN["rows"]}
TRAJ, MC, T = GOLDEN["trajectories"], 4, GOLDEN["steps"]


@pytest.fixture(scope="module")
def rmse_of():
    import torch

    from paper_2109_13504_amd import mgp
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    n = GOLDEN["n"]
    truth, z = inputs.sir_truth(T, TRAJ)
    zr = np.repeat(z, MC, axis=0)
    x0 = inputs.sir_initial_particles_torch(TRAJ * MC, n, torch.device("cuda:0"))
    cache = {}

    def run(variant, B):
        if (variant, B) not in cache:
            f = mgp.SirFilter(TRAJ * MC, n, T, variant=variant, B=B, seed=2021)
            f.set_measurements(zr)
            f.reset(x0)
            f.run()
            est, bs, st = f.results()
            f.close()
            assert (st == 0).all() and (bs == (B if B else 1)).all()
            e = est.reshape(TRAJ, MC, T) - truth[:, None, 1:]
            cache[(variant, B)] = float(np.sqrt(np.mean(e * e, axis=1)).mean(axis=1).mean())
        return cache[(variant, B)]

    return run


ROWS = sorted(PAPER, key=lambda k: (k[1], k[0]))


@pytest.mark.parametrize("variant,B", ROWS, ids=[f"{v}-B{b}" for v, b in ROWS])
def test_rmse_near_table2(rmse_of, variant, B):
    """Every resampler row of Table 2 (four variants x B = 16, 32, 64)."""
    got = rmse_of(variant, B)
    assert abs(got - PAPER[(variant, B)]) < 0.3, (variant, B, got, PAPER[(variant, B)])


@pytest.mark.parametrize("B", [16, 32, 64])
def test_table2_orderings(rmse_of, B):
    """The orderings Table 2 shows at each B: C1 with 128-byte partitions is
    the worst by a clear margin (0.12-0.15 in the table), while Megopolis,
    Metropolis and C2 lie within 0.015 of one another."""
    c1 = rmse_of("c1", B)
    others = [rmse_of(v, B) for v in ("megopolis", "metropolis", "c2")]
    assert c1 > max(others) + 0.05, (B, c1, others)
    assert max(others) - min(others) < 0.05, (B, others)


@pytest.mark.parametrize("variant", ["megopolis", "metropolis", "c1", "c2"])
def test_table2_rmse_falls_with_B(rmse_of, variant):
    """Each resampler's RMSE falls from B = 16 to 32 to 64 in Table 2, by
    0.017-0.075 per doubling; the runs here share their seeds across B."""
    r16, r32, r64 = (rmse_of(variant, b) for b in (16, 32, 64))
    assert r16 > r32 - 0.005 and r32 > r64 - 0.01 and r16 > r64, (variant, r16, r32, r64)


UNBIASED = {r["method"]: r["rmse"] for r in GOLDEN["unbiased"]}


@pytest.mark.parametrize("method", ["multinomial", "systematic"])
def test_unbiased_rows_near_table2(rmse_of, method):
    """Table 2's unbiased rows: stage 2 by multinomial (Algorithm 7) or
    systematic (Algorithm 8) resampling through the prefix sum."""
    got = rmse_of(method, 0)
    assert abs(got - UNBIASED[method]) < 0.3, (method, got, UNBIASED[method])


def test_unbiased_rows_orderings(rmse_of):
    """Table 2: the unbiased methods have the lowest RMSE (2.944), below C1 at
    every B (3.10-3.17) and below the B = 16 rows (3.04-3.17), and Megopolis
    approaches them as B grows (2.948 at B = 64)."""
    for m in ("multinomial", "systematic"):
        u = rmse_of(m, 0)
        for B in (16, 32, 64):
            assert u < rmse_of("c1", B) - 0.05, (m, B)
        assert u < rmse_of("megopolis", 16) - 0.02, m
        assert abs(u - rmse_of("megopolis", 64)) < 0.05, m


def test_b_study_claims(rmse_of):
    """Section 7's B study (its figures; no printed values): RMSE falls with
    B with diminishing returns, C1 with 128-byte partitions needs about
    B = 25 to match what Megopolis reaches at B = 10, and C1 stays above
    Megopolis at equal B."""
    mego = [rmse_of("megopolis", b) for b in (5, 10, 20, 40)]
    assert mego[0] > mego[1] > mego[2] > mego[3]
    assert mego[0] - mego[1] > mego[2] - mego[3]
    assert abs(rmse_of("c1", 25) - rmse_of("megopolis", 10)) < 0.06
    assert rmse_of("c1", 10) > rmse_of("megopolis", 10) + 0.05


def test_epsilon_mode_mean_B_near_paper_baseline():
    """Section 7 derives B per step from eq. (bcalc) with epsilon = 0.1 and
    reports an average of 30 iterations at 2^20 particles."""
    import torch

    from paper_2109_13504_amd import mgp
    n = GOLDEN["n"]
    _, z = inputs.sir_truth(T, TRAJ)
    zr = np.repeat(z, MC, axis=0)
    x0 = inputs.sir_initial_particles_torch(TRAJ * MC, n, torch.device("cuda:0"))
    f = mgp.SirFilter(TRAJ * MC, n, T, variant="megopolis", B=0, epsilon=0.1, seed=2021)
    f.set_measurements(zr)
    f.reset(x0)
    f.run()
    _, bs, st = f.results()
    f.close()
    assert (st == 0).all() and (bs >= 1).all()
    assert 20.0 < bs.mean() < 40.0, bs.mean()
    print("mean B at epsilon = 0.1:", bs.mean())
