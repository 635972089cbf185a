"""Tiny problems (N <= 8) where the full distribution of the ancestor vector
can be enumerated exactly, compared with the oracle over many seeds by a
chi-square test.

The acceptance probability of a step k -> j is the fraction of the 2^24
u levels with fl32(u w_k) <= w_j (the product form of the ratio test in
Algorithms 2-5). Metropolis: particles run independent chains with uniform
candidates. C1: the group's partition p is uniform and fixed, then candidates
are uniform inside it. Megopolis: given the offsets the candidate of particle
i at step b is (i + o_b) mod N (N <= 16), and the particles' u draws are
independent, so the joint law is the average over all offset sequences of a
product of per-particle laws.
"""
import itertools

import numpy as np
import pytest
from scipy.stats import chisquare

import oracle
from helpers import chain_marginal, fixed_candidate_step, megopolis_index_small, transition_matrix

W4 = np.array([0.15, 0.6, 0.35, 1.0], dtype=np.float32)
W5 = np.array([0.0, 0.4, 1.0, 0.05, 0.7], dtype=np.float32)


def _encode(anc, n):
    code = 0
    for a in anc:
        code = code * n + int(a)
    return code


def _chi2(observed_codes, probs):
    n_cells = probs.size
    obs = np.bincount(observed_codes, minlength=n_cells).astype(float)
    exp = probs * obs.sum()
    # pool cells with small expectation into one
    small = exp < 5
    o = np.concatenate([obs[~small], [obs[small].sum()]]) if small.any() else obs
    e = np.concatenate([exp[~small], [exp[small].sum()]]) if small.any() else exp
    keep = e > 0
    assert np.all(o[~keep] == 0), "outcome with zero probability observed"
    return chisquare(o[keep], e[keep]).pvalue


def _joint_independent(marginals):
    n = marginals[0].size
    probs = np.ones(1)
    for m in marginals:
        probs = np.outer(probs, m).ravel()
    return probs.reshape([n] * len(marginals)).ravel()


@pytest.mark.parametrize("w,B", [(W4, 3), (W5, 4)])
def test_metropolis_joint_law(w, B):
    n = w.size
    T = transition_matrix(w)
    probs = _joint_independent([chain_marginal(T, i, B) for i in range(n)])
    codes = [_encode(oracle.resample(w, "metropolis", B, s), n) for s in range(30000)]
    assert _chi2(np.array(codes), probs) > 1e-4


@pytest.mark.parametrize("w,B", [(W4, 3), (W4, 6), (W5, 3)])
def test_megopolis_joint_law(w, B):
    n = w.size
    probs = np.zeros(n ** n)
    for offs in itertools.product(range(n), repeat=B):
        margs = []
        for i in range(n):
            v = np.zeros(n)
            v[i] = 1.0
            for o in offs:
                v = fixed_candidate_step(v, w, megopolis_index_small(i, o, n))
            margs.append(v)
        probs += _joint_independent(margs)
    probs /= n ** B
    assert abs(probs.sum() - 1) < 1e-9
    codes = [_encode(oracle.resample(w, "megopolis", B, s), n) for s in range(30000)]
    assert _chi2(np.array(codes), probs) > 1e-4


def test_megopolis_and_metropolis_share_marginals_but_not_joint():
    # same per-particle law (uniform candidates), different joint law:
    # under Megopolis two particles never propose the same index at one step
    w, B = W4, 3
    n = w.size
    T = transition_matrix(w)
    runs = 30000
    anc = np.array([oracle.resample(w, "megopolis", B, s) for s in range(runs)])
    for i in range(n):
        obs = np.bincount(anc[:, i], minlength=n)
        assert chisquare(obs, chain_marginal(T, i, B) * runs).pvalue > 1e-4


@pytest.mark.parametrize("w,B", [(W4, 3), (np.array([0.2, 1.0, 0.5, 0.9, 0.3, 0.05], np.float32), 2)])
def test_c1_joint_law(w, B):
    """8-byte partitions (N_w = 2): the single group draws one partition p
    (uniform over ceil(N/2)) and every particle runs a chain whose candidates
    are uniform inside partition p."""
    n = w.size
    nw = 2
    n_part = (n + nw - 1) // nw
    probs = np.zeros(n ** n)
    for p in range(n_part):
        support = np.arange(p * nw, min(n, (p + 1) * nw))
        Tp = transition_matrix(w, support)
        probs += _joint_independent([chain_marginal(Tp, i, B) for i in range(n)])
    probs /= n_part
    codes = [_encode(oracle.resample(w, "c1", B, s, partition_bytes=8), n) for s in range(30000)]
    assert _chi2(np.array(codes), probs) > 1e-4


def test_c2_marginal_law():
    """C2 redraws the partition every step, so with equal partitions each
    step's candidate is uniform over all N: the Metropolis marginal."""
    w, B = W4, 4
    n = w.size
    T = transition_matrix(w)
    runs = 30000
    anc = np.array([oracle.resample(w, "c2", B, s, partition_bytes=8) for s in range(runs)])
    for i in range(n):
        obs = np.bincount(anc[:, i], minlength=n)
        assert chisquare(obs, chain_marginal(T, i, B) * runs).pvalue > 1e-4


def test_exact_law_detects_a_planted_mistake():
    """The enumeration is sharp enough to reject a chain with a plausible
    slip: comparing against the starting particle's weight w_i instead of the
    current ancestor's w_k."""
    w, B = W4, 3
    n = w.size
    T = transition_matrix(w)
    probs = _joint_independent([chain_marginal(T, i, B) for i in range(n)])
    g = np.random.Generator(np.random.PCG64(0))
    runs = 8000
    j = g.integers(0, n, (runs, n, B))
    u = ((g.integers(0, 1 << 24, (runs, n, B)) + 1) / 2 ** 24).astype(np.float32)
    k = np.tile(np.arange(n), (runs, 1))
    for b in range(B):
        stale = (u[:, :, b] * w[np.arange(n)][None, :]) <= w[j[:, :, b]]
        k = np.where(stale, j[:, :, b], k)
    codes = np.array([_encode(row, n) for row in k])
    assert _chi2(codes, probs) < 1e-6
