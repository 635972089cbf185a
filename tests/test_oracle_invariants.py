"""Pins for the accept loop on weight vectors where the outcome is known in
closed form: uniform weights, a single nonzero weight, two-level weights
(where the recurrence of Section 4.1 is exact), and the expected offspring
that Metropolis, C2 and Megopolis share (Sections 4.1, 6.1)."""
import numpy as np
import pytest

import oracle
from helpers import chain_marginal, recurrence_P, transition_matrix
from oracle.metrics import QualityAccumulator, offspring
from paper_2109_13504_amd import inputs

VARIANTS = ["metropolis", "c1", "c2", "megopolis"]


@pytest.mark.parametrize("variant", VARIANTS)
def test_uniform_weights_accept_every_candidate(variant):
    n, B = 256, 9
    w = inputs.uniform_weights(n, 0.7)
    anc, acc = oracle.resample(w, variant, B, 17, return_accepts=True)
    assert acc == n * B
    for i in range(0, n, 7):
        j, _ = oracle.trace(n, variant, B, 17, i)
        assert anc[i] == j[-1]


@pytest.mark.parametrize("n", [64, 4096, 12])
def test_megopolis_uniform_weights_gives_permutation(n):
    # every offset maps particles one-to-one (N % 32 == 0, or one segment)
    w = inputs.uniform_weights(n)
    for seed in range(5):
        anc = oracle.resample(w, "megopolis", 7, seed)
        assert np.array_equal(np.sort(anc), np.arange(n))


def test_metropolis_uniform_weights_mse():
    # anc_i i.i.d. uniform: offspring multinomial(N, 1/N), E[SE] = N (1 - 1/N)
    n = 512
    w = inputs.uniform_weights(n)
    q = QualityAccumulator(w)
    for s in range(400):
        q.add(oracle.resample(w, "metropolis", 3, s))
    assert abs(q.mse_over_n() - (1 - 1 / n)) < 5 * q.mse_over_n_stderr()


@pytest.mark.parametrize("variant", VARIANTS)
def test_single_nonzero_weight(variant):
    """From a zero weight every candidate is accepted (u * 0 <= w_j); from the
    only nonzero weight every other candidate is rejected (u > 0). So particle
    i ends at p iff p is among its candidates, else at its last candidate."""
    n, B, p = 256, 12, 77
    w = inputs.single_spike_weights(n, p)
    anc = oracle.resample(w, variant, B, 5)
    for i in range(n):
        j, _ = oracle.trace(n, variant, B, 5, i)
        expect = p if (i == p or p in j) else j[-1]
        assert anc[i] == expect, (i, j)


def test_megopolis_single_weight_offspring_bounded_by_B_plus_one():
    # each offset exposes particle p to exactly one other particle
    n, B, p = 1024, 20, 300
    w = inputs.single_spike_weights(n, p)
    for s in range(10):
        anc = oracle.resample(w, "megopolis", B, s)
        assert 1 <= np.sum(anc == p) <= B + 1


def test_metropolis_single_weight_collapse_probability():
    n, B, p, runs = 128, 30, 9, 300
    w = inputs.single_spike_weights(n, p)
    frac = np.mean([np.mean(oracle.resample(w, "metropolis", B, s) == p) for s in range(runs)])
    expect = 1 / n + (1 - 1 / n) * (1 - (1 - 1 / n) ** B)
    sd = np.sqrt(expect * (1 - expect) / (n * runs))
    assert abs(frac - expect) < 5 * sd


@pytest.mark.parametrize("variant", ["metropolis", "c2", "megopolis"])
def test_two_level_weights_follow_recurrence(variant):
    """w_p = 1, others c with c 2^24 an integer: the recurrence
    P_B = 1/N + P_{B-1}(1 - E(w)/w_p) of Section 4.1 is exact, and
    E[#{i != p: anc_i = p}] = (N - 1) P_B."""
    n, p, c, B, runs = 1024, 17, 0.25, 10, 120
    w = inputs.two_level_weights(n, p, c)
    ratio = (1 + (n - 1) * c) / n
    PB = recurrence_P(n, ratio, B)
    counts = []
    for s in range(runs):
        anc = oracle.resample(w, variant, B, 1000 + s)
        counts.append(np.sum(anc == p) - (anc[p] == p))
    counts = np.array(counts, dtype=float)
    expect = (n - 1) * PB
    se = counts.std(ddof=1) / np.sqrt(runs)
    assert abs(counts.mean() - expect) < 5 * se + 1e-9, (counts.mean(), expect, se)


def test_two_level_recurrence_equals_exact_chain():
    n, p, c, B = 16, 4, 0.25, 10
    w = inputs.two_level_weights(n, p, c)
    T = transition_matrix(w)
    exact = chain_marginal(T, 0, B)[p]
    assert abs(exact - recurrence_P(n, (1 + (n - 1) * c) / n, B)) < 1e-14


@pytest.mark.parametrize("variant", ["metropolis", "c2", "megopolis"])
def test_expected_offspring_matches_exact_chain(variant):
    """Every candidate of Metropolis, C2 (N_w | N) and Megopolis (N % 32 == 0)
    is marginally uniform (Section 4.1), so E[offspring] = 1^T T^B for the
    one-step matrix T: the reason their bias contributions agree (Section 6.1)."""
    n, B, runs = 256, 6, 400
    w = inputs.gaussian_weights(n, 2.0, 5)
    T = transition_matrix(w)
    TB = np.linalg.matrix_power(T, B)
    expect = TB.sum(axis=0)
    offs = np.array([offspring(oracle.resample(w, variant, B, 7000 + s), n) for s in range(runs)], float)
    mean = offs.mean(axis=0)
    sd = offs.std(axis=0, ddof=1) / np.sqrt(runs)
    z = (mean - expect) / np.maximum(sd, 1e-3)
    assert np.max(np.abs(z)) < 5.5
    # aggregate check: chi-square-like statistic close to its mean n
    assert np.sum(z ** 2) < n + 6 * np.sqrt(2 * n)
