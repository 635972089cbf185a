"""Pins for the candidate-index maps (Algorithms 2-5) against the properties
the paper states for them (Sections 3, 3.1, 4): Megopolis gives every offset
a unique index (a bijection of the particles), reads one aligned 32-weight
segment per 32 threads, and reduces to the misaligned cyclic shift when the
array fits one segment; C1/C2 candidates stay inside one partition per group.
"""
import numpy as np
import pytest

import oracle
from helpers import megopolis_index_small


def mego_map(n, o):
    return np.array([oracle.megopolis_index(i, o, n) for i in range(n)])


@pytest.mark.parametrize("n", [32, 64, 96, 160, 1024])
def test_megopolis_map_is_bijection_when_n_multiple_of_32(n):
    offs = range(n) if n <= 160 else np.random.Generator(np.random.PCG64(1)).integers(0, n, 40)
    for o in offs:
        j = mego_map(n, int(o))
        assert j.min() >= 0 and j.max() < n
        assert np.unique(j).size == n, (n, o)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 13, 16])
def test_megopolis_map_is_cyclic_shift_for_single_segment(n):
    for o in range(n):
        for i in range(n):
            assert oracle.megopolis_index(i, o, n) == megopolis_index_small(i, o, n)


@pytest.mark.parametrize("n", [17, 31, 33, 100, 1000])
def test_megopolis_map_stays_in_range_for_ragged_n(n):
    # The literal formula (with mod N) is used for any N; it is not a
    # bijection when N is not a multiple of 32, but always a valid index.
    for o in range(0, n, max(1, n // 37)):
        j = mego_map(n, o)
        assert j.min() >= 0 and j.max() < n


def test_megopolis_map_aligned_segment_rotation():
    # particles of one 32-wide segment read one aligned 32-wide segment,
    # rotated by o mod 32 (the wrapped sequential pattern)
    n = 4096
    for o in [0, 1, 31, 32, 33, 1000, 4095]:
        j = mego_map(n, o)
        for seg in range(0, n, 32):
            js = j[seg:seg + 32]
            base = js.min()
            assert base % 32 == 0
            assert sorted(js - base) == list(range(32))
            assert js[0] - base == o % 32


def _lines_per_wave(j_rows, n, wave=64, line_bytes=128):
    """distinct 128-byte lines touched per 64-particle wave, per iteration"""
    per = []
    for jb in j_rows:
        for s in range(0, n, wave):
            per.append(np.unique((jb[s:s + wave] * 4) // line_bytes).size)
    return np.array(per)


def _all_j(n, variant, B, seed, partition_bytes=128):
    rows = np.empty((B, n), dtype=np.int64)
    for i in range(n):
        j, _ = oracle.trace(n, variant, B, seed, i, partition_bytes=partition_bytes)
        rows[:, i] = j
    return rows


def test_cache_lines_per_wave_by_variant():
    """Transactions per warp (Sections 3, 3.1, 4): Megopolis touches exactly
    the 2 aligned 128-byte lines a 64-wide wave covers; C1/C2 with 128-byte
    partitions touch one line per 32-thread group; Metropolis touches close to
    one line per thread."""
    n, B = 4096, 6
    mego = _lines_per_wave(_all_j(n, "megopolis", B, 21), n)
    assert np.all(mego == 2)
    for v in ("c1", "c2"):
        lines = _lines_per_wave(_all_j(n, v, B, 21, 128), n)
        assert lines.max() <= 2
    metro = _lines_per_wave(_all_j(n, "metropolis", B, 21), n)
    # 64 uniform draws over 128 lines: E[distinct] = 128 (1 - (127/128)^64) ~ 50.5
    assert 45 < metro.mean() < 56


def test_c1_partition_fixed_per_group_and_c2_redrawn():
    n, B, ps = 2048, 12, 256
    nw = ps // 4
    rows1 = _all_j(n, "c1", B, 5, ps)
    rows2 = _all_j(n, "c2", B, 5, ps)
    for g in range(0, n, 32):
        p1 = rows1[:, g:g + 32] // nw
        assert np.unique(p1).size == 1  # one partition for the whole group, all b
        p2 = rows2[:, g:g + 32] // nw
        for b in range(B):
            assert np.unique(p2[b]).size == 1  # one partition per group per b
    # C2's partition changes across iterations
    changes = [np.unique(rows2[:, g] // nw).size for g in range(0, n, 32)]
    assert np.mean(changes) > 6


def test_c1_c2_ragged_last_partition():
    # N not a multiple of N_w: the last partition is cut at N
    n, ps = 1000, 128  # N_w = 32, 31.25 partitions -> 32 partitions, last has 8
    for v in ("c1", "c2"):
        rows = _all_j(n, v, 8, 77, ps)
        assert rows.min() >= 0 and rows.max() < n
    # with enough draws the short partition [992, 1000) is reached
    hits = 0
    for s in range(60):
        j, _ = oracle.trace(n, "c2", 40, s, 0, partition_bytes=ps)
        hits += np.sum(j >= 992)
    assert hits > 0


def test_metropolis_candidates_uniform():
    from scipy.stats import chisquare
    n = 50
    js = np.concatenate([oracle.trace(n, "metropolis", 40, 3, i)[0] for i in range(n)]
                        + [oracle.trace(n, "metropolis", 40, 4, i)[0] for i in range(n)])
    assert chisquare(np.bincount(js, minlength=n)).pvalue > 1e-4
