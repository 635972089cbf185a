"""Megopolis with 64-wide segments (the wavefront width of gfx950; the
paper's segment is its 32-thread warp). Pinned by facts of the index map and
of the law it induces, not by retyping it:
  - for N <= 32 the map is the cyclic shift (i + o) mod N;
  - for N a multiple of 64 every offset gives a bijection;
  - the 64 candidates of an aligned 64-particle group fill exactly two
    aligned 128-byte lines;
  - for N <= 32 each particle's candidate is uniform over the inputs at
    every step (o_b is uniform), so its ancestor follows the Metropolis chain
    marginal (checked at N = 20, where the 32-wide map is not a shift);
  - for N <= 16 both segment widths are the cyclic shift: identical results."""
import numpy as np
import pytest
from scipy.stats import chisquare

import oracle
from helpers import chain_marginal, transition_matrix


@pytest.mark.parametrize("n", [1, 5, 17, 20, 32])
def test_small_n_is_cyclic_shift(n):
    for i in range(n):
        for o in range(n):
            assert oracle.megopolis_index(i, o, n, segment=64) == (i + o) % n


@pytest.mark.parametrize("n", [64, 128, 320])
def test_bijection_when_64_divides_n(n):
    for o in range(n):
        js = {oracle.megopolis_index(i, o, n, segment=64) for i in range(n)}
        assert js == set(range(n))


def test_two_lines_per_aligned_group():
    n = 4096
    for o in (0, 1, 31, 32, 63, 64, 100, 4000, 4095):
        for g in range(0, n, 64):
            lines = {(oracle.megopolis_index(i, o, n, segment=64) * 4) // 128 for i in range(g, g + 64)}
            assert len(lines) == 2, (o, g, lines)


def test_ancestor_law_at_n20_is_the_uniform_candidate_chain():
    rng = np.random.default_rng(8)
    w = rng.random(20).astype(np.float32)
    n, B, seeds = 20, 3, 20000
    T = transition_matrix(w)
    anc = np.array([oracle.resample_m(w, n, "megopolis", B, s, segment=64) for s in range(seeds)])
    for i in (0, 3, 17, 19):
        p = chain_marginal(T, i, B)
        obs = np.bincount(anc[:, i], minlength=n).astype(float)
        keep = p * seeds >= 5
        o = np.concatenate([obs[keep], [obs[~keep].sum()]])
        e = np.concatenate([p[keep], [p[~keep].sum()]]) * seeds
        assert chisquare(o[e > 0], e[e > 0]).pvalue > 1e-4, i


@pytest.mark.parametrize("n", [3, 9, 16])
def test_equal_to_32_wide_segments_for_n_up_to_16(n):
    w = np.random.default_rng(n).random(n).astype(np.float32)
    for s in range(50):
        np.testing.assert_array_equal(oracle.resample_m(w, n, "megopolis", 5, s, segment=64),
                                      oracle.resample(w, "megopolis", 5, s))


def test_other_segments_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.resample_m(np.ones(8, np.float32), 8, "megopolis", 2, 1, segment=48)
