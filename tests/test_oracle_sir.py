"""Pins of the oracle's SIR application (Section 7, Algorithm 6) to things
other than itself: the noise against the normal law (KS test), the
prediction against the model's conditional mean and variance, the weight
against scipy's normal density, the estimate against math.fsum, the whole
filter against an independent numpy SIR filter with multinomial resampling,
and the mean B at epsilon = 0.1 against the baseline the paper reports."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2109_13504_amd import inputs


def model_mean(c, t):
    """E[x_t | x_{t-1} = c] of eq. (predict-end2end)."""
    return c / 2.0 + 25.0 * c / (1.0 + c * c) + 8.0 * math.cos(1.2 * t)


def test_noise_is_standard_normal():
    e = np.array([oracle.sir_normal(11, 3, i, 5) for i in range(20000)])
    assert stats.kstest(e, "norm").pvalue > 1e-3
    assert abs(e.mean()) < 5 / math.sqrt(e.size)
    assert abs(e.var() - 1.0) < 5 * math.sqrt(2.0 / e.size)
    # other steps and runs are independent draws
    e2 = np.array([oracle.sir_normal(11, 3, i, 6) for i in range(20000)])
    e3 = np.array([oracle.sir_normal(11, 4, i, 5) for i in range(20000)])
    assert abs(np.corrcoef(e, e2)[0, 1]) < 5 / math.sqrt(e.size)
    assert abs(np.corrcoef(e, e3)[0, 1]) < 5 / math.sqrt(e.size)
    # Box-Muller pairs (particles 2m, 2m+1): uncorrelated, and the squared
    # radius e_2m^2 + e_2m+1^2 is chi-square with 2 degrees of freedom
    a, b = e[0::2], e[1::2]
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(a.size)
    assert stats.kstest(a * a + b * b, "expon", args=(0, 2)).pvalue > 1e-3
    # the two pairs of one generator call are independent of each other
    assert abs(np.corrcoef(e[0::4], e[2::4])[0, 1]) < 5 / math.sqrt(e.size / 4)


@pytest.mark.parametrize("c,t", [(-3.0, 1), (0.5, 2), (2.0, 7), (10.0, 40), (0.0, 13)])
def test_prediction_law(c, t):
    """From x_bar = c for every particle, x_t ~ N(model_mean(c, t), 10)."""
    n = 40000
    x, _ = oracle.sir_predict_update(np.full(n, c, dtype=np.float32), t, 0.0, 5, 2)
    m = float(np.float32(c))
    mu = model_mean(m, t)
    assert abs(x.mean() - mu) < 5 * math.sqrt(10.0 / n)
    assert abs(x.var() - 10.0) < 5 * 10.0 * math.sqrt(2.0 / n)
    assert stats.kstest((x - mu) / math.sqrt(10.0), "norm").pvalue > 1e-3


def test_weight_is_gaussian_likelihood():
    """w = p(z | x) of eq. (update-end2end) without its 1/sqrt(2 pi) factor."""
    rng = np.random.default_rng(4)
    xbar = rng.normal(0, 6, 5000).astype(np.float32)
    for z in (0.3, 4.0, 17.5):
        x, w = oracle.sir_predict_update(xbar, 3, z, 9, 0)
        ref = stats.norm.pdf(z, loc=x.astype(np.float64) ** 2 / 20.0, scale=1.0) * math.sqrt(2 * math.pi)
        np.testing.assert_allclose(w, ref.astype(np.float32), rtol=2.4e-7, atol=1e-44)
        assert w.max() > 0


def test_mean_is_exact_sum_over_n():
    rng = np.random.default_rng(5)
    for n in (1, 7, 4096, 100003):
        v = (rng.normal(0, 10, n) * (1 + rng.integers(0, 1000, n))).astype(np.float32)
        ref = math.fsum(v.astype(np.float64).tolist()) / n
        assert abs(oracle.mean(v) - ref) <= 2 * n * 2.0 ** -53 * np.abs(v.astype(np.float64)).mean() + 1e-300


def numpy_sir(x0, z, rng):
    """An independent bootstrap filter: same model, multinomial resampling."""
    xb = x0.astype(np.float64)
    est = []
    for t in range(1, len(z)):
        xp = xb / 2 + 25 * xb / (1 + xb * xb) + 8 * np.cos(1.2 * t) + rng.normal(0, np.sqrt(10), xb.size)
        w = np.exp(-0.5 * (z[t] - xp * xp / 20) ** 2)
        xb = xp[rng.choice(xb.size, xb.size, p=w / w.sum())]
        est.append(xb.mean())
    return np.array(est)


def rmse(est_runs, truth):
    """RMSE of Section 7: per step over the runs, averaged over the steps."""
    e = np.asarray(est_runs) - truth[None, :]
    return float(np.mean(np.sqrt(np.mean(e * e, axis=0))))


@pytest.mark.parametrize("variant,B", [("megopolis", 32), ("metropolis", 32), ("c2", 32)])
def test_filter_matches_multinomial_sir(variant, B):
    """On the same trajectories, the oracle's filter and a numpy bootstrap
    filter reach the same RMSE (Table 2: the resamplers differ by a few
    hundredths at B >= 32), and both beat the prior alone by far."""
    T, N = 100, 2048
    truth, z = inputs.sir_truth(T, 2)
    for tr in range(2):
        ours, ref, prior = [], [], []
        for run in range(3):
            x0 = inputs.sir_initial_particles(N, run + 10 * tr)
            est, bs, st, _ = oracle.sir_filter(x0, z[tr], variant, B, 77, run + 10 * tr)
            assert (st == 0).all() and (bs == B).all()
            ours.append(est)
            ref.append(numpy_sir(x0, z[tr], np.random.default_rng(run)))
            # the prediction alone, without the update (the measurement
            # ignored): uniform weights
            xb = x0.copy()
            pe = []
            for t in range(1, T + 1):
                xb, _ = oracle.sir_predict_update(xb, t, 0.0, 77, run)
                pe.append(oracle.mean(xb))
            prior.append(pe)
        r_ours, r_ref, r_prior = rmse(ours, truth[tr, 1:]), rmse(ref, truth[tr, 1:]), rmse(prior, truth[tr, 1:])
        assert abs(r_ours - r_ref) < 0.3, (tr, r_ours, r_ref)
        assert r_ours < 0.75 * r_prior, (tr, r_ours, r_prior)


def test_epsilon_mode_mean_B_near_paper_baseline():
    """Section 7 derives B per step from eq. (bcalc) with epsilon = 0.1 and
    reports an average of 30 iterations; with the same model the oracle's
    per-step B averages in that range."""
    T, N = 100, 2048
    _, z = inputs.sir_truth(T, 4)
    means = []
    for tr in range(4):
        x0 = inputs.sir_initial_particles(N, 50 + tr)
        _, bs, st, _ = oracle.sir_filter(x0, z[tr], "megopolis", 0, 3, tr, epsilon=0.1)
        assert (st == 0).all() and (bs >= 1).all()
        means.append(bs.mean())
    assert 15.0 < np.mean(means) < 50.0, means


def test_degenerate_step_keeps_predicted_particles():
    """A measurement no particle can explain makes every fp32 weight 0; the
    step then keeps the predicted particles and reports MGP_EWEIGHTS."""
    T, N = 5, 1024
    _, z = inputs.sir_truth(T, 1)
    z = z[0].copy()
    z[3] = 1e6
    x0 = inputs.sir_initial_particles(N, 0)
    _, _, _, xbar2 = oracle.sir_filter(x0, z, "megopolis", 8, 21, 0, steps=2)
    x3, w3 = oracle.sir_predict_update(xbar2, 3, float(z[3]), 21, 0)
    assert (w3 == 0).all()
    est, bs, st, xbar3 = oracle.sir_filter(x0, z, "megopolis", 8, 21, 0, steps=3)
    assert st.tolist() == [0, 0, oracle.EWEIGHTS] and bs[2] == 0
    np.testing.assert_array_equal(xbar3, x3)
    assert est[2] == oracle.mean(x3)
    # the filter goes on from there
    est5, _, st5, _ = oracle.sir_filter(x0, z, "megopolis", 8, 21, 0)
    assert st5[3] == 0 and st5[4] == 0 and np.isfinite(est5).all()
