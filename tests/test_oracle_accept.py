"""Pins for the oracle's acceptance rules (CPU only)."""

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import accept, assign, balance, diagnose, prep


def test_paper_planning_counts(golden):
    g = golden["planning_counts"]
    for N, k in zip(g["draws"], g["accepted"]):
        assert accept.quantile_count(g["q"], N) == k


def test_workload_counts():
    assert accept.quantile_count(0.01, 184756) == 1848
    assert accept.quantile_count(0.01, 200000) == 2000
    assert accept.quantile_count(1.2e-5, 100_000_000) == 1200
    assert accept.quantile_count(0.01, 100_000) == 1000
    assert accept.quantile_count(1.0, 7) == 7
    assert accept.quantile_count(1e-9, 7) == 1


@given(st.integers(1, 300), st.data())
@settings(max_examples=100, deadline=None)
def test_quantile_equals_sort_when_distinct(N, data):
    rng = np.random.default_rng(data.draw(st.integers(0, 10 ** 6)))
    M = rng.permutation(N).astype(np.float64) + 1.0       # distinct, gaps >> eps
    keys = rng.choice(10 ** 9, size=N, replace=False).astype(np.uint64)
    k = data.draw(st.integers(1, N))
    got = accept.accept_quantile(keys, M, k)
    want = np.sort(keys[np.argsort(M)[:k]])
    np.testing.assert_array_equal(got, want)


def test_tie_rule_orders_near_equal_values_by_key():
    keys = np.array([50, 10, 40, 20, 30, 60], dtype=np.uint64)
    t = 5.0
    M = np.array([1.0, t, t * (1 + 3e-11), t * (1 - 2e-11), 9.0, 0.5])
    # L = {1.0, 0.5} (keys 50, 60); E = {keys 10, 40, 20}; k = 4 -> two from E: 10, 20
    got = accept.accept_quantile(keys, M, 4)
    np.testing.assert_array_equal(got, np.array([10, 20, 50, 60], dtype=np.uint64))
    # outside the eps band the order is by M again
    M2 = M.copy()
    M2[2] = t * (1 - 1e-6)
    got = accept.accept_quantile(keys, M2, 4)
    np.testing.assert_array_equal(got, np.array([10, 40, 50, 60], dtype=np.uint64))


@given(st.integers(2, 200), st.data())
@settings(max_examples=100, deadline=None)
def test_count_is_exactly_k_with_ties(N, data):
    rng = np.random.default_rng(data.draw(st.integers(0, 10 ** 6)))
    M = rng.integers(0, 5, size=N).astype(np.float64)      # heavy exact ties
    keys = rng.choice(10 ** 9, size=N, replace=False).astype(np.uint64)
    k = data.draw(st.integers(1, N))
    got = accept.accept_quantile(keys, M, k)
    assert len(got) == k
    assert len(set(got.tolist())) == k
    # every accepted value <= every rejected value
    acc = np.isin(keys, got)
    if acc.all() or not acc.any():
        return
    assert M[acc].max() <= M[~acc].min()


def test_threshold():
    keys = np.arange(6, dtype=np.uint64)
    M = np.array([3.0, 1.0, 2.0, 2.0, 5.0, 0.0])
    np.testing.assert_array_equal(accept.accept_threshold(keys, M, 2.0), [1, 2, 3, 5])


def test_accepted_mean_matches_truncated_chi2():
    # Appendix A part C: E[M | M <= a] = d v_a(d) on the chi^2 scale (Gaussian covariates,
    # d << n); the q-quantile acceptance approximates the threshold rule.
    n, d, N, q = 2000, 5, 20000, 0.1
    X = np.random.default_rng(8).standard_normal((n, d))
    P = prep.prepare(X, n // 2)
    keys = np.arange(N, dtype=np.uint64)
    W = assign.mc_assignments_batch(23, keys, n, n // 2)
    M = balance.mahalanobis_batch(X, W, P["S_lam"])
    k = accept.quantile_count(q, N)
    acc = accept.accept_quantile(keys, M, k)
    Macc = M[acc.astype(np.int64)]
    want = diagnose.expected_M_accept(d, q)
    assert abs(Macc.mean() - want) < 5 * Macc.std() / np.sqrt(k) + 0.03 * want


def test_bad_q():
    with pytest.raises(ValueError):
        accept.quantile_count(0.0, 10)
    with pytest.raises(ValueError):
        accept.quantile_count(1.5, 10)
