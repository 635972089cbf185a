"""Pins of the oracle's prefix-sum resamplers, the unbiased comparison
methods of Section 6.5 and Table 2: multinomial (Algorithm 7) and
systematic (Algorithm 8) resampling.

What fixes them without an implementation to compare against:
  - the fixed-point weights q_i = floor(w_i 2^K) against exact rational
    arithmetic, and the prefix sums against Python's exact integers;
  - multinomial: the offspring vector is Multinomial(N, q / S): the ancestor
    law by a chi-square test on a tiny problem, E[SE] = sum N p (1 - p) and no
    bias over many runs;
  - systematic: every offspring count is floor(N p_j) or ceil(N p_j) (the
    defining property of systematic resampling), the ancestors are
    nondecreasing, the mean offspring is N p_j over random u, and equal
    weights give the identity;
  - both: zero weights are never chosen, a single nonzero weight takes every
    output, and the thresholds come from the (pinned) Philox words of their
    own tags.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.metrics import QualityAccumulator
from paper_2109_13504_amd import inputs
from scipy import stats as sstats

METHODS = ["multinomial", "systematic"]


def _weights_mix(n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    w = g.gamma(0.7, 1.0, n).astype(np.float32)
    w[g.integers(0, n, max(1, n // 10))] = 0.0
    w[g.integers(0, n, 3)] = np.float32(1e-30)  # far below the fixed-point resolution: q = 0
    w[g.integers(0, n, 2)] = np.float32(3e-38)
    return w


@pytest.mark.parametrize("n", [1, 7, 1000, 4097])
def test_fixed_point_is_exact(n):
    w = _weights_mix(n, n) if n > 1 else np.array([0.3], np.float32)
    incl, K = oracle.prefix_sum(w)
    wmax = float(w.max())
    m, E = math.frexp(wmax)
    assert K == 62 - math.ceil(math.log2(n)) - E if n > 1 else K == 62 - E
    total = 0
    for j, v in enumerate(w):
        q = math.floor(Fraction(float(v)) * Fraction(2) ** K)
        assert oracle.prefix_fixed(v, K) == q
        total += q
        assert int(incl[j]) == total
    assert total < 2**62
    # the largest weight keeps about 62 - log2 n bits
    assert oracle.prefix_fixed(wmax, K) >= 2 ** (61 - math.ceil(math.log2(max(n, 2))))


def test_prefix_rejects_invalid_weights():
    for bad in (np.nan, np.inf, -1.0):
        w = np.ones(10, np.float32)
        w[3] = bad
        with pytest.raises(oracle.OracleError):
            oracle.resample_prefix(w, "systematic", 1)
    with pytest.raises(oracle.OracleError):
        oracle.resample_prefix(np.zeros(5, np.float32), "multinomial", 1)


def test_thresholds_from_their_philox_words():
    n, S = 1000, 987654321987
    for i in (0, 1, 999):
        x = oracle.philox4x32_10([0, 6, 3, i], [5, 0])
        r = int(x[0]) | (int(x[1]) << 32)
        assert oracle.prefix_threshold("multinomial", S, n, 5, 3, i) == (r * S) >> 64
    x = oracle.philox4x32_10([0, 7, 3, 0], [5, 0])
    r = int(x[0]) | (int(x[1]) << 32)
    ut = float(r >> 11) * 2.0**-53
    for i in (0, 17, 999):
        t = oracle.prefix_threshold("systematic", S, n, 5, 3, i)
        exact = (Fraction(i) + Fraction(ut)) * Fraction(S, n)
        assert abs(t - math.floor(exact)) <= 1
        assert 0 <= t < S


def test_multinomial_ancestor_law_tiny():
    """N = 5 with exactly representable weights: each output's ancestor is
    drawn from q / S (chi-square over 4000 calls x 5 outputs)."""
    w = np.array([0.125, 0.0, 0.5, 0.25, 0.125], np.float32)
    incl, K = oracle.prefix_sum(w)
    p = np.diff(np.concatenate([[0], incl.astype(object)])).astype(float) / float(incl[-1])
    counts = np.zeros(5)
    for s in range(4000):
        a = oracle.resample_prefix(w, "multinomial", 1000 + s)
        counts += np.bincount(a, minlength=5)
    assert counts[1] == 0
    keep = p > 0
    chi2 = sstats.chisquare(counts[keep], counts.sum() * p[keep])
    assert chi2.pvalue > 1e-3, chi2


def test_multinomial_offspring_moments():
    n = 300
    w = inputs.gaussian_weights(n, 2.0, 4)
    incl, _ = oracle.prefix_sum(w)
    q = np.diff(np.concatenate([[0], incl.astype(object)])).astype(float)
    p = q / q.sum()
    acc = QualityAccumulator(q)  # expected offspring N q / S
    for s in range(2000):
        acc.add(oracle.resample_prefix(w, "multinomial", s, stream_id=2))
    expect = float(np.sum(n * p * (1 - p))) / n
    assert abs(acc.mse_over_n() - expect) < 5 * acc.mse_over_n_stderr()
    var = acc.variance_sum()
    assert abs(acc.bias_sq_debiased()) < 5 * var / acc.k / math.sqrt(n / 4)


@pytest.mark.parametrize("n", [10, 333, 4096])
def test_systematic_offspring_are_floor_or_ceil(n):
    for seed in range(20):
        w = _weights_mix(n, 50 + seed) if seed % 2 else inputs.gaussian_weights(n, 3.0, seed)
        incl, _ = oracle.prefix_sum(w)
        S = int(incl[-1])
        q = np.diff(np.concatenate([[0], incl.astype(object)]))
        a = oracle.resample_prefix(w, "systematic", seed, stream_id=seed)
        assert np.all(np.diff(a) >= 0)
        o = np.bincount(a, minlength=n)
        for j in range(n):
            lo = (n * int(q[j])) // S
            hi = -((-n * int(q[j])) // S)
            assert lo <= o[j] <= hi, (n, seed, j, o[j], lo, hi)


def test_systematic_mean_offspring_unbiased():
    n = 64
    w = _weights_mix(n, 3)
    incl, _ = oracle.prefix_sum(w)
    q = np.diff(np.concatenate([[0], incl.astype(object)])).astype(float)
    expect = n * q / q.sum()
    mean = np.zeros(n)
    K = 4000
    for s in range(K):
        mean += np.bincount(oracle.resample_prefix(w, "systematic", s), minlength=n)
    mean /= K
    # o_j = floor(N p_j) + Bernoulli(frac(N p_j)): sd of the mean <= 0.5 / sqrt(K)
    assert np.max(np.abs(mean - expect)) < 5 * 0.5 / math.sqrt(K)


def test_systematic_equal_weights_identity():
    for n in (1, 5, 1000, 4099):
        a = oracle.resample_prefix(np.full(n, 0.37, np.float32), "systematic", 9)
        np.testing.assert_array_equal(a, np.arange(n))


@pytest.mark.parametrize("method", METHODS)
def test_single_nonzero_weight_takes_every_output(method):
    n = 777
    w = np.zeros(n, np.float32)
    w[401] = 2.5
    assert (oracle.resample_prefix(w, method, 3) == 401).all()


@pytest.mark.parametrize("method", METHODS)
def test_zero_weights_never_chosen(method):
    n = 5000
    w = _weights_mix(n, 8)
    incl, _ = oracle.prefix_sum(w)
    q = np.diff(np.concatenate([[0], incl.astype(object)]))
    a = oracle.resample_prefix(w, method, 12)
    assert (q[a] > 0).all()
    assert a.min() >= 0 and a.max() < n
