"""Pins for the oracle's conditional randomization test (CPU only)."""

from fractions import Fraction
from math import comb

import numpy as np

from oracle import assign, frt


def small_case(n=10, n1=5, seed=0):
    rng = np.random.default_rng(seed)
    W = assign.exact_assignments(n, n1)
    Y = rng.standard_normal(n) * 3 + W[17] * 1.5
    return W, Y


def test_dim_sums_to_zero_over_all_assignments():
    W, Y = small_case()
    Z = [Fraction(float(y)) for y in Y]
    assert sum(frt.dim_exact(w, Z) for w in W) == 0


def test_dim_variance_over_all_assignments():
    # Var_w DiM = n/(n1 n0) * s_y^2 with s_y^2 the sample variance (denominator n - 1)
    n, n1 = 9, 4
    W = assign.exact_assignments(n, n1)
    Y = [Fraction(int(v)) for v in np.random.default_rng(1).integers(-50, 50, n)]
    D = [frt.dim_exact(w, Y) for w in W]
    mean = sum(D) / len(D)
    var = sum((x - mean) ** 2 for x in D) / len(D)
    ybar = sum(Y) / n
    s2 = sum((y - ybar) ** 2 for y in Y) / (n - 1)
    assert var == Fraction(n, n1 * (n - n1)) * s2


def test_fast_form_equals_definition():
    W, Y = small_case()
    taus = [0.0, 0.5, -1.25, 3.0, 1e-3]
    r = frt.rand_test(W, 17, Y, taus)
    assert r["counts"] == frt.rand_test_definition(W, 17, Y, taus)


def test_p_is_one_at_tau_hat():
    W, Y = small_case(seed=2)
    r = frt.rand_test(W, 17, Y, [0.0])
    r2 = frt.rand_test(W, 17, Y, [r["tau_hat_exact"]])
    assert r2["counts"] == [len(W)]


def test_p_lower_bound_and_large_tau():
    # |T_obs(tau0)| grows like |tau0| n1 n0 / (n1 n0) with the largest slope any draw can
    # have; only w_obs itself and (n1 = n0) its complement keep up, so far out on the grid
    # the count is 2 here (the complement is among all assignments).
    W, Y = small_case(seed=3)
    r = frt.rand_test(W, 17, Y, [1e6, -1e6])
    assert r["counts"] == [2, 2]
    K = len(W)
    assert all(c / K >= 1 / K for c in r["counts"])
    # Monte Carlo subset without the complement: count 1, p = 1/K
    sub = W[[17, 3, 40, 100]]
    r = frt.rand_test(sub, 0, Y, [1e6])
    assert r["counts"] == [1]


def test_quantized_equals_unquantized():
    rng = np.random.default_rng(4)
    n, n1, K = 30, 15, 200
    W = assign.mc_assignments_batch(5, np.arange(K, dtype=np.uint64), n, n1)
    Y = rng.standard_normal(n) + W[0]
    taus = list(np.linspace(-2, 2, 9))
    assert frt.rand_test(W, 0, Y, taus)["counts"] == frt.rand_test_unquantized(W, 0, Y, taus)


def test_quantization_shift_bounds():
    for n in [20, 100, 1000, 2000]:
        Y = np.random.default_rng(n).standard_normal(n) * 7
        s = frt.quantization_shift(Y, n)
        Yq = frt.quantize(Y, s)
        m = max(abs(v) for v in Yq)
        assert 2 * n * n * m <= 2 ** 63
        assert m >= 2 ** 61 // (4 * n * n)        # uses most of the range


def test_min_p_paper_numbers(golden):
    g = golden["planning_counts"]
    for K, pmin in zip(g["accepted"], g["min_p"]):
        assert abs(1 / K - pmin) < 1e-12


def test_interval():
    taus = [-2, -1, 0, 1, 2]
    assert frt.interval(taus, [0.01, 0.2, 0.9, 0.3, 0.04]) == dict(lo=-1.0, hi=1.0, contiguous=True)
    assert frt.interval(taus, [0.01, 0.2, 0.01, 0.3, 0.04])["contiguous"] is False


def test_exact_count_small():
    assert comb(10, 5) == 252
