"""M != N resampling (Section 8: for D-PMC-style use the Megopolis offsets
range over the number of inputs). Reading taken: output i in [0, M) starts
its chain at input i mod N and draws its own u and j; candidates range over
the N inputs. Pinned on tiny problems by the exact joint law of the M
ancestors, enumerated as in test_oracle_exact (Metropolis: independent
chains from i mod N with uniform candidates; Megopolis, N <= 16: the cyclic
shift (i mod N + o_b) mod N averaged over all offset sequences), and by
consistency with the M = N resampler."""
import itertools

import numpy as np
import pytest

import oracle
from helpers import chain_marginal, fixed_candidate_step, megopolis_index_small, transition_matrix
from test_oracle_exact import W4, W5, _chi2, _encode, _joint_independent


@pytest.mark.parametrize("w,m,B", [(W4, 6, 3), (W4, 3, 4), (W5, 7, 2)])
def test_metropolis_m_outputs_joint_law(w, m, B):
    n = w.size
    T = transition_matrix(w)
    probs = _joint_independent([chain_marginal(T, i % n, B) for i in range(m)])
    codes = [_encode(oracle.resample_m(w, m, "metropolis", B, s), n) for s in range(30000)]
    assert _chi2(np.array(codes), probs) > 1e-4


@pytest.mark.parametrize("w,m,B", [(W4, 6, 3), (W4, 2, 4), (W5, 8, 2)])
def test_megopolis_m_outputs_joint_law(w, m, B):
    n = w.size
    probs = np.zeros(n ** m)
    for offs in itertools.product(range(n), repeat=B):
        margs = []
        for i in range(m):
            v = np.zeros(n)
            v[i % n] = 1.0
            for o in offs:
                v = fixed_candidate_step(v, w, megopolis_index_small(i % n, o, n))
            margs.append(v)
        probs += _joint_independent(margs)
    probs /= n ** B
    assert abs(probs.sum() - 1) < 1e-9
    codes = [_encode(oracle.resample_m(w, m, "megopolis", B, s), n) for s in range(30000)]
    assert _chi2(np.array(codes), probs) > 1e-4


@pytest.mark.parametrize("variant", ["megopolis", "metropolis", "c1", "c2"])
def test_m_equal_n_is_the_resampler_and_prefixes_agree(variant):
    w = np.random.default_rng(3).random(1000).astype(np.float32)
    ref = oracle.resample(w, variant, 9, 17, stream_id=2)
    np.testing.assert_array_equal(oracle.resample_m(w, 1000, variant, 9, 17, stream_id=2), ref)
    # fewer outputs: the first m chains; more outputs: the first n are the M = N ones
    np.testing.assert_array_equal(oracle.resample_m(w, 613, variant, 9, 17, stream_id=2), ref[:613])
    more = oracle.resample_m(w, 2345, variant, 9, 17, stream_id=2)
    np.testing.assert_array_equal(more[:1000], ref)
    assert more.min() >= 0 and more.max() < 1000


def test_m_offspring_mean_is_m_times_normalised_weight():
    """With many steps every output's ancestor follows the normalised
    weights, so the mean offspring count of input j is M w_j / sum(w)."""
    w = np.array([0.1, 0.5, 0.2, 1.0, 0.05, 0.3, 0.7, 0.4], dtype=np.float32)
    n, m, B, runs = w.size, 50, 60, 400
    counts = np.zeros(n)
    for s in range(runs):
        counts += np.bincount(oracle.resample_m(w, m, "metropolis", B, 1000 + s), minlength=n)
    expect = m * runs * w / w.sum()
    # multinomial standard deviation per cell
    sd = np.sqrt(m * runs * (w / w.sum()) * (1 - w / w.sum()))
    assert np.all(np.abs(counts - expect) < 5 * sd + 1), (counts, expect)


def test_bad_m_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.resample_m(W4, 0, "metropolis", 3, 1)
