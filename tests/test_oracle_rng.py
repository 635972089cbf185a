"""Pins for the oracle's random streams: Philox4x32-10 against an independent
implementation, and the u / index maps against their exact definitions."""
import numpy as np
import pytest

import oracle
from helpers import philox_reference


def test_philox_matches_rocrand_engine():
    ref = philox_reference()
    if ref is None:
        pytest.skip("hipcc not available to build the rocRAND reference")
    g = np.random.Generator(np.random.PCG64(4242))
    cases = [([0, 0, 0, 0], [0, 0]), ([1, 0, 0, 0], [0, 0]), ([0, 0, 0, 1], [0, 0]),
             ([0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF], [0xFFFFFFFF, 0xFFFFFFFF])]
    for _ in range(300):
        c = g.integers(0, 2**32, 4, dtype=np.uint64).astype(np.uint32)
        c[1] &= 0x3FFFFFFF  # the engine reaches word 1 through a 64-bit offset of 4 per block
        k = g.integers(0, 2**32, 2, dtype=np.uint64).astype(np.uint32)
        cases.append((c, k))
    for c, k in cases:
        np.testing.assert_array_equal(oracle.philox4x32_10(c, k), ref(c, k), err_msg=f"ctr={c} key={k}")


def test_philox_avalanche():
    # flipping one counter bit changes about half of the 128 output bits
    base = oracle.philox4x32_10([5, 6, 7, 8], [9, 10])
    flips = []
    for word in range(4):
        for bit in (0, 13, 31):
            c = np.array([5, 6, 7, 8], dtype=np.uint32)
            c[word] ^= np.uint32(1 << bit)
            out = oracle.philox4x32_10(c, [9, 10])
            flips.append(sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(base, out)))
    assert 48 <= np.mean(flips) <= 80


def test_u_on_exact_grid_in_half_open_unit_interval():
    us = np.array([oracle.draw_u(7, 3, i, b) for i in range(50) for b in range(23)], dtype=np.float32)
    assert us.min() > 0.0 and us.max() <= 1.0
    m = us.astype(np.float64) * 2**24
    np.testing.assert_array_equal(m, np.round(m))  # multiples of 2^-24


def test_u_stream_words_layout():
    """u_b of particle i comes from Philox call (b // 5, tag 0, stream, i): the
    first four from the top 24 bits of each word, the fifth from the low
    bytes of words 0, 1, 2."""
    seed, stream, i = 0x1234_5678_9ABC_DEF0, 11, 77
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for q in range(3):
        x = [int(v) for v in oracle.philox4x32_10([q, 0, stream, i], key)]
        ms = [x[0] >> 8, x[1] >> 8, x[2] >> 8, x[3] >> 8,
              (x[0] & 255) | ((x[1] & 255) << 8) | ((x[2] & 255) << 16)]
        for r in range(5):
            assert float(oracle.draw_u(seed, stream, i, 5 * q + r)) == (ms[r] + 1) / 2**24


def test_u_uniformity_chi_square():
    from scipy.stats import chisquare
    us = np.array([oracle.draw_u(99, 0, i, b) for i in range(400) for b in range(50)])
    counts, _ = np.histogram(us, bins=20, range=(0, 1))
    assert chisquare(counts).pvalue > 1e-4


def test_offsets_uniform_over_range_and_shared():
    from scipy.stats import chisquare
    n = 40
    o = oracle.offsets(5, 0, n, 20000)
    assert o.min() >= 0 and o.max() < n
    assert chisquare(np.bincount(o, minlength=n)).pvalue > 1e-4
    # offsets depend on (seed, stream) only, not on anything per particle
    np.testing.assert_array_equal(o[:100], oracle.offsets(5, 0, n, 100))
    assert not np.array_equal(o[:100], oracle.offsets(5, 1, n, 100))


def test_offset_index_map_is_mulhi():
    seed, stream, n = 3, 2, 1000003
    key = [seed, 0]
    for b in range(12):
        x = int(oracle.philox4x32_10([b // 4, 2, stream, 0], key)[b % 4])
        assert oracle.offsets(seed, stream, n, b + 1)[b] == (x * n) >> 32
