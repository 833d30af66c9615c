"""Pins for the oracle's assignment generation (CPU only)."""

import itertools
from math import comb

import numpy as np
from hypothesis import given, settings, strategies as st
from scipy import stats

from oracle import assign


def brute_smallest(u, n1):
    # rank of unit i = number of units that come before it in (u, index) order
    n = len(u)
    rank = [sum(1 for k in range(n) if (u[k], k) < (u[i], i)) for i in range(n)]
    return sorted(i for i in range(n) if rank[i] < n1)


@given(st.lists(st.integers(0, 7), min_size=2, max_size=40), st.data())
@settings(max_examples=200, deadline=None)
def test_smallest_set_matches_brute_force(u, data):
    n1 = data.draw(st.integers(1, len(u) - 1))
    assert assign.smallest_set(u, n1) == brute_smallest(u, n1)


def test_batch_matches_scalar():
    seed = 0x0123456789ABCDEF
    for n, n1 in [(20, 10), (100, 50), (257, 100), (1000, 500)]:
        keys = [0, 1, 2 ** 32 + 5, 2 ** 64 - 1]
        Wb = assign.mc_assignments_batch(seed, keys, n, n1)
        for row, b in zip(Wb, keys):
            np.testing.assert_array_equal(row, assign.mc_assignment(seed, b, n, n1))
            assert row.sum() == n1


def test_complete_randomization_is_uniform():
    # every one of the C(6,3) = 20 subsets equally likely; marginals n1/n
    n, n1, N = 6, 3, 40000
    W = assign.mc_assignments_batch(99, np.arange(N, dtype=np.uint64), n, n1)
    codes = (W * (1 << np.arange(n))).sum(axis=1)
    _, counts = np.unique(codes, return_counts=True)
    assert len(counts) == comb(n, n1)
    assert stats.chisquare(counts).pvalue > 1e-4
    marg = W.mean(axis=0)
    assert np.all(np.abs(marg - n1 / n) < 5 * np.sqrt(0.25 / N))


def test_colex_small_known_order():
    # combinatorial number system: rank = C(i1, 1) + C(i2, 2)
    order = [[0, 1], [0, 2], [1, 2], [0, 3], [1, 3], [2, 3]]
    assert [assign.colex_unrank(r, 4, 2) for r in range(6)] == order


def test_colex_bijection():
    n, n1 = 11, 4
    seen = set()
    for r in range(comb(n, n1)):
        t = assign.colex_unrank(r, n, n1)
        assert assign.colex_rank(t) == r
        seen.add(tuple(t))
    assert seen == set(itertools.combinations(range(n), n1))


def test_pack_roundtrip():
    rng = np.random.default_rng(3)
    for n in [1, 31, 32, 33, 100, 1000]:
        W = rng.integers(0, 2, size=(5, n)).astype(np.uint8)
        P = assign.pack_bits(W)
        assert P.shape == (5, (n + 31) // 32)
        np.testing.assert_array_equal(assign.unpack_bits(P, n), W)
        # bit i % 32 of word i // 32
        i = n - 1
        assert ((int(P[0, i // 32]) >> (i % 32)) & 1) == W[0, i]
