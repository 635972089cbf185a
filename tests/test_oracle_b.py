"""Pins for the reduction and the iteration count B (eq. (bcalc), eq.
(proposition), Section 4.1 and Section 6.3)."""
import math

import numpy as np
import pytest

import oracle
from helpers import gaussian_B_closed_form
from paper_2109_13504_amd import inputs


def test_closed_form_gaussian_B_values():
    # Section 6.3's E(w) and max w give r = exp(-y^2/4)/sqrt(2)
    assert [gaussian_B_closed_form(y) for y in range(5)] == [4, 6, 16, 60, 354]


@pytest.mark.parametrize("y", [0, 1, 2, 3, 4])
def test_sample_B_close_to_population_B(y):
    w = inputs.gaussian_weights(1 << 20, y, 0)
    B, raw, clamped = oracle.B_from_weights(w, 0.01)
    assert not clamped
    assert abs(B - gaussian_B_closed_form(y)) <= max(1, round(0.02 * B)), (B, raw)


@pytest.mark.parametrize("n,c,eps", [(1024, 0.25, 0.01), (100, 0.5, 0.05), (4096, 0.001, 0.01),
                                     (7, 0.9, 1e-6)])
def test_B_is_minimal_solution_of_bias_bound(n, c, eps):
    """Section 4.1 derives (1 - E(w)/w_p)^B = eps; the chosen B is the
    smallest integer with (1 - r)^B <= eps."""
    w = inputs.two_level_weights(n, 3, c)
    B, raw, _ = oracle.B_from_weights(w, eps)
    r = (1.0 + (n - 1) * float(np.float32(c))) / n
    assert (1.0 - r) ** B <= eps * (1 + 1e-12)
    if B > 1:
        assert (1.0 - r) ** (B - 1) > eps


def test_B_uniform_weights_is_one():
    B, raw, _ = oracle.B_from_weights(inputs.uniform_weights(1000, 0.3), 0.01)
    assert B == 1


def test_B_eps_one_is_one():
    w = inputs.gaussian_weights(1000, 2.0)
    assert oracle.B_from_weights(w, 1.0)[0] == 1


def test_B_clamped_to_b_max():
    w = inputs.single_spike_weights(1 << 12, 5)  # r = 1/N: raw ~ N log(1/eps)
    B, raw, clamped = oracle.B_from_weights(w, 0.01, b_max=1000)
    assert clamped and B == 1000 and raw > 1000
    B2, raw2, clamped2 = oracle.B_from_weights(w, 0.01)
    # single nonzero weight: r = 1/N, B = ceil(log eps / log(1 - 1/N)) ~ N ln(100)
    assert not clamped2 and abs(B2 - math.log(100) * (1 << 12)) < 3


def test_B_rejects_bad_eps():
    with pytest.raises(oracle.OracleError):
        oracle.choose_B(1.0, 1.0, 10, 0.0)
    with pytest.raises(oracle.OracleError):
        oracle.choose_B(1.0, 1.0, 10, 1.5)


def test_reduce_sum_against_exact_sum():
    w = inputs.gaussian_weights(200001, 1.5, 3)
    st = oracle.reduce(w)
    assert st.status == 0
    exact = math.fsum(float(v) for v in w)
    assert abs(st.w_sum - exact) <= 1e-12 * exact
    assert st.w_max == float(w.max())


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf, -1e-30])
def test_reduce_flags_invalid_weights(bad):
    w = inputs.gaussian_weights(100, 0.0)
    w[37] = bad
    assert oracle.reduce(w).status == oracle.EWEIGHTS


def test_reduce_flags_all_zero():
    assert oracle.reduce(np.zeros(64, np.float32)).status == oracle.EWEIGHTS


def test_reduce_accepts_negative_zero():
    w = inputs.gaussian_weights(100, 0.0)
    w[3] = -0.0
    assert oracle.reduce(w).status == 0
