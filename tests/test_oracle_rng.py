"""Pins of the oracle's random numbers: Philox4x64-10 and the pair draw.

The oracle's Philox is checked against numpy's independent Philox4x64-10
(numpy advances its 256-bit counter before producing a block, so block c
is numpy's first output when started from counter c - 1).
"""
import numpy as np
import pytest
from scipy.stats import chisquare


def numpy_block(key, ctr):
    c = [int(x) for x in ctr]
    # counter - 1 with borrow across the 256-bit counter
    i = 0
    while i < 4:                # all-zero counter wraps to all ones
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = 2**64 - 1
        i += 1
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    return g.random_raw(4)


@pytest.mark.parametrize("key,ctr", [
    ((1, 0), (0, 0, 0, 0)),
    ((1, 0), (5, 17, 0, 0)),
    ((0xDEADBEEF, 1), (0, 123456789, 0, 0)),
    ((2**64 - 1, 3), (2**63, 2**40, 0, 0)),
    ((7, 2), (1, 0, 0, 0)),
])
def test_philox_matches_numpy(oracle, key, ctr):
    got = oracle.philox_block(key[0], key[1], ctr)
    want = numpy_block(key, ctr)
    assert np.array_equal(got, want)


def test_draw_layout_is_a_counter_stream(oracle):
    # draws 0..11 of sample 9 on stream 1 = three consecutive blocks
    seed, stream, sample = 42, 1, 9
    g = np.random.Philox(key=np.array([seed, stream], dtype=np.uint64),
                         counter=np.array([2**64 - 1, sample - 1, 0, 0], dtype=np.uint64))
    want = g.random_raw(12)
    got = np.array([oracle.draw(seed, stream, sample, j) for j in range(12)], dtype=np.uint64)
    assert np.array_equal(got, want)


def test_pair_is_uniform_over_ordered_pairs(oracle):
    n = 7
    counts = np.zeros((n, n))
    N = 84000
    for i in range(N):
        s, t = oracle.pair(3, 0, i, n)
        assert s != t and 0 <= s < n and 0 <= t < n
        counts[s, t] += 1
    obs = counts[~np.eye(n, dtype=bool)]
    assert chisquare(obs).pvalue > 1e-4


def test_pair_two_vertices(oracle):
    seen = {oracle.pair(1, 0, i, 2) for i in range(64)}
    assert seen == {(0, 1), (1, 0)}
