"""Pins for the oracle's balance statistic M (CPU only)."""

from math import comb

import numpy as np
import pytest
from scipy import stats

from oracle import assign, balance, prep


def all_M(X, n1, ridge_rel=0.0):
    P = prep.prepare(X, n1, ridge_rel)
    W = assign.exact_assignments(X.shape[0], n1)
    return W, balance.mahalanobis_batch(X, W, P["S_lam"]), P


def test_mean_over_all_assignments_is_d():
    # E_w[M] = (n1 n0 / n) tr(S^-1 Cov_w(Delta)) and Cov_w(Delta) = n/(n1 n0) S exactly
    # under complete randomization, so the mean over all C(n, n1) assignments is d.
    X = np.random.default_rng(0).standard_normal((12, 3))
    _, M, _ = all_M(X, 6)
    assert abs(M.mean() - 3.0) < 1e-12


def test_mean_with_ridge_is_trace():
    X = np.random.default_rng(1).standard_normal((11, 4))
    _, M, P = all_M(X, 4, ridge_rel=0.3)
    want = np.trace(np.linalg.solve(P["S_lam"], P["S"]))
    assert abs(M.mean() - want) < 1e-12
    assert want < 4.0


def test_range_and_complement_symmetry():
    X = np.random.default_rng(2).standard_normal((12, 5))
    W, M, P = all_M(X, 6)
    assert M.min() >= 0 and M.max() <= 12 - 1 + 1e-9
    Mc = balance.mahalanobis_batch(X, 1 - W, P["S_lam"])
    np.testing.assert_allclose(Mc, M, rtol=1e-12, atol=1e-12)


def test_affine_invariance():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((30, 4))
    A = rng.standard_normal((4, 4)) + 3 * np.eye(4)
    b = rng.standard_normal(4) * 10
    W = assign.mc_assignments_batch(5, np.arange(50, dtype=np.uint64), 30, 13)
    M1 = balance.mahalanobis_batch(X, W, prep.prepare(X, 13)["S_lam"])
    Y = X @ A + b
    M2 = balance.mahalanobis_batch(Y, W, prep.prepare(Y, 13)["S_lam"])
    np.testing.assert_allclose(M1, M2, rtol=1e-9)


def test_whitened_sum_form_agrees():
    # M = n/(n1 n0) || L^-1 sum_{i in T} (X_i - mu) ||^2, the whitened form of the
    # Appendix A remark, with the centring that makes the control sum redundant.
    rng = np.random.default_rng(4)
    X = rng.standard_normal((40, 6))
    P = prep.prepare(X, 17, ridge_rel=0.05)
    W = assign.mc_assignments_batch(11, np.arange(30, dtype=np.uint64), 40, 17)
    G = W @ (X - P["mu"])
    Z = np.linalg.solve(P["L"], G.T).T
    alt = 40 / (17 * 23) * (Z ** 2).sum(axis=1)
    np.testing.assert_allclose(balance.mahalanobis_batch(X, W, P["S_lam"]), alt, rtol=1e-12)


def test_chi2_scale():
    # Section 2.2: M ~ (1/n_T + 1/n_C) chi^2_d on the paper's scale for whitened Gaussian
    # covariates, i.e. chi^2_d on the scale reported here.
    n, d, N = 2000, 10, 3000
    X = np.random.default_rng(5).standard_normal((n, d))
    P = prep.prepare(X, n // 2)
    W = assign.mc_assignments_batch(17, np.arange(N, dtype=np.uint64), n, n // 2)
    M = balance.mahalanobis_batch(X, W, P["S_lam"])
    assert stats.kstest(M, stats.chi2(d).cdf).pvalue > 1e-3
    assert abs(M.mean() - d) < 4 * np.sqrt(2 * d / N)


def test_singular_detected():
    X = np.random.default_rng(6).standard_normal((10, 12))
    with pytest.raises(prep.SingularCovariance):
        prep.prepare(X, 5, 0.0)
    P = prep.prepare(X, 5, 1e-2)          # ridge makes it positive definite
    assert np.all(np.diag(P["L"]) > 0)


def test_rank_deficient_pinv_is_constant():
    # Without a ridge and with d >= n - 1, the pseudo-inverse makes M = n - 1 for every
    # draw (why a ridge is needed for the n = d workloads).
    n = 15
    X = np.random.default_rng(7).standard_normal((n, n))
    mu, S = prep.covariance(X)
    W = assign.mc_assignments_batch(3, np.arange(20, dtype=np.uint64), n, 7)
    d = W @ X / 7 - (1 - W) @ X / 8
    M = 7 * 8 / n * np.einsum("bj,jk,bk->b", d, np.linalg.pinv(S), d)
    np.testing.assert_allclose(M, n - 1, rtol=1e-8)


def test_exact_enumeration_count():
    assert comb(20, 10) == 184756


# ---- diagonal (standardise-only) metric
def all_M_metric(X, n1, metric, ridge_rel=0.0):
    P = prep.prepare(X, n1, ridge_rel, metric)
    W = assign.exact_assignments(X.shape[0], n1)
    return W, balance.mahalanobis_batch(X, W, P["S_lam"]), P


def test_diagonal_reduces_to_mahalanobis_for_one_covariate():
    X = np.random.default_rng(20).standard_normal((12, 1))
    _, Md, _ = all_M_metric(X, 5, "diagonal")
    _, Mm, _ = all_M_metric(X, 5, "mahalanobis")
    np.testing.assert_allclose(Md, Mm, rtol=1e-12)


def test_diagonal_equals_mahalanobis_for_orthogonal_columns():
    # centred columns of a Hadamard design are orthogonal, so S is diagonal
    H = np.array([[1, 1, 1, 1], [1, -1, 1, -1], [1, 1, -1, -1], [1, -1, -1, 1]], dtype=float)
    X = np.kron(H, np.ones((3, 1)))[:, 1:] * np.array([1.0, 2.5, 0.3])
    _, Md, _ = all_M_metric(X, 6, "diagonal")
    _, Mm, _ = all_M_metric(X, 6, "mahalanobis")
    np.testing.assert_allclose(Md, Mm, rtol=1e-12, atol=1e-12)


def test_diagonal_mean_over_all_assignments():
    # each standardised mean difference has variance exactly 1 / scale over all assignments
    X = np.random.default_rng(21).standard_normal((12, 4)) @ np.random.default_rng(22).standard_normal((4, 4))
    _, M, P = all_M_metric(X, 6, "diagonal")
    assert abs(M.mean() - 4.0) < 1e-12
    _, M, P = all_M_metric(X, 6, "diagonal", ridge_rel=0.5)
    S = np.diag(P["S"])
    assert abs(M.mean() - np.sum(S / (S + P["lam"]))) < 1e-12


def test_diagonal_scaling_invariant_not_rotation_invariant():
    rng = np.random.default_rng(23)
    X = rng.standard_normal((12, 3))
    _, M, _ = all_M_metric(X, 6, "diagonal")
    _, Ms, _ = all_M_metric(X * np.array([3.0, 0.1, 7.0]) + 5.0, 6, "diagonal")
    np.testing.assert_allclose(Ms, M, rtol=1e-10)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    _, Mr, _ = all_M_metric(X @ Q, 6, "diagonal")
    _, Mm, _ = all_M_metric(X, 6, "mahalanobis")
    _, Mmr, _ = all_M_metric(X @ Q, 6, "mahalanobis")
    np.testing.assert_allclose(Mmr, Mm, rtol=1e-10)
    assert np.max(np.abs(Mr - M)) > 1e-3


def test_diagonal_constant_column_is_singular():
    X = np.random.default_rng(24).standard_normal((10, 3))
    X[:, 1] = 2.0
    with pytest.raises(prep.SingularCovariance):
        prep.prepare(X, 5, 0.0, "diagonal")


# ---- per-column criterion: the largest squared standardised mean difference
def all_M_max(X, n1, ridge_rel=0.0):
    P = prep.prepare(X, n1, ridge_rel, "max_smd")
    W = assign.exact_assignments(X.shape[0], n1)
    return W, balance.max_smd_batch(X, W, np.diag(P["S_lam"])), P


def test_max_smd_one_covariate_is_the_two_sample_statistic():
    # with d = 1 the largest term is the only term: the textbook two-sample z^2 (Mahalanobis),
    # with and without a ridge
    X = np.random.default_rng(30).standard_normal((12, 1)) * 3.0 + 1.0
    for ridge in (0.0, 0.4):
        _, Mx, _ = all_M_max(X, 5, ridge)
        _, Mm, _ = all_M_metric(X, 5, "mahalanobis", ridge)
        np.testing.assert_allclose(Mx, Mm, rtol=1e-12)


def test_max_smd_between_max_and_sum():
    # max_j z_j^2 <= sum_j z_j^2 <= d max_j z_j^2 for every assignment, and the sum is the
    # standardise-only M
    X = np.random.default_rng(31).standard_normal((12, 4)) @ np.random.default_rng(32).standard_normal((4, 4))
    W, Mx, _ = all_M_max(X, 6)
    _, Md, _ = all_M_metric(X, 6, "diagonal")
    assert np.all(Mx <= Md * (1 + 1e-12)) and np.all(Md <= 4 * Mx * (1 + 1e-12))
    # and each column alone gives a lower bound that is attained by the largest column
    per_col = np.stack([all_M_metric(X[:, [j]], 6, "diagonal")[1] for j in range(4)])
    np.testing.assert_allclose(Mx, per_col.max(axis=0), rtol=1e-12)


def test_max_smd_duplicated_and_rescaled_columns():
    # a column repeated with another scale and offset changes nothing (per-column
    # standardisation); permuting the columns changes nothing; M(w) = M(1 - w)
    X = np.random.default_rng(33).standard_normal((11, 3))
    W, Mx, _ = all_M_max(X, 4)
    X2 = np.column_stack([X[:, 2], X[:, 0] * -7.0 + 3.0, X[:, 1], X[:, 0] * 0.01])
    _, Mx2, _ = all_M_max(X2, 4)
    np.testing.assert_allclose(Mx2, Mx, rtol=1e-10)
    P = prep.prepare(X, 5, 0.0, "max_smd")
    W5 = assign.exact_assignments(11, 5)
    W6 = 1 - W5
    np.testing.assert_allclose(balance.max_smd_batch(X, W5, np.diag(P["S_lam"])),
                               balance.max_smd_batch(X, W6, np.diag(P["S_lam"])), rtol=1e-12)


def test_max_smd_distribution_is_max_of_chi2_1():
    # independent Gaussian columns: M_max ~ max of d chi^2_1, P(M_max <= t) = F_1(t)^d
    n, d, N = 2000, 5, 3000
    X = np.random.default_rng(34).standard_normal((n, d))
    P = prep.prepare(X, n // 2, 0.0, "max_smd")
    W = assign.mc_assignments_batch(19, np.arange(N, dtype=np.uint64), n, n // 2)
    Mx = balance.max_smd_batch(X, W, np.diag(P["S_lam"]))
    assert stats.kstest(Mx, lambda t: stats.chi2(1).cdf(t) ** d).pvalue > 1e-3
    # the sum of the terms would follow chi^2_d instead: clearly rejected
    assert stats.kstest(Mx, stats.chi2(d).cdf).pvalue < 1e-6
