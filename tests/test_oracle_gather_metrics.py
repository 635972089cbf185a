"""Pins for the particle copy (x_bar_i = x_k, Algorithms 2-5) and for the
quality measures of Section 5.1."""
import numpy as np
import pytest

import oracle
from oracle.metrics import QualityAccumulator, offspring
from paper_2109_13504_amd import inputs


@pytest.mark.parametrize("d", [1, 3, 4, 8, 16])
def test_gather_equals_fancy_indexing(d):
    st = inputs.random_states(1000, d, 3)
    anc = np.random.Generator(np.random.PCG64(d)).integers(0, 1000, 777).astype(np.int32)
    np.testing.assert_array_equal(oracle.gather(st, anc), st[anc])


def test_gather_rejects_out_of_range():
    st = inputs.random_states(10, 2, 1)
    with pytest.raises(oracle.OracleError):
        oracle.gather(st, np.array([0, 10], np.int32))
    with pytest.raises(oracle.OracleError):
        oracle.gather(st, np.array([-1], np.int32))


def test_offspring_counts_sum_to_n():
    anc = np.array([3, 3, 0, 1, 3], np.int32)
    np.testing.assert_array_equal(offspring(anc, 5), [1, 1, 0, 3, 0])


def test_mse_of_multinomial_resampling_closed_form():
    """Multinomial resampling: offspring ~ Multinomial(N, w_bar), so
    E[SE] = sum_i N w_bar_i (1 - w_bar_i) and the bias is zero."""
    n = 300
    w = inputs.gaussian_weights(n, 2.0, 4).astype(np.float64)
    wb = w / w.sum()
    g = np.random.Generator(np.random.PCG64(8))
    q = QualityAccumulator(w)
    for _ in range(3000):
        q.add(np.repeat(np.arange(n), g.multinomial(n, wb)))
    expect = np.sum(n * wb * (1 - wb)) / n
    assert abs(q.mse_over_n() - expect) < 5 * q.mse_over_n_stderr()
    assert q.bias_contribution() < 0.05
