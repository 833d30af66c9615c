"""Pins for the design closed forms against the paper's printed numbers (CPU only)."""

import numpy as np
from scipy import integrate, stats

from oracle import balance, diagnose, prep


def test_v_a_rule_of_thumb(golden):
    g = golden["v_a_q001"]
    for d, want in g["values"].items():
        assert round(diagnose.v_a(int(d), g["q"]), g["decimals"]) == want


def test_rmse_drop(golden):
    g = golden["rmse_drop_pct"]
    for d, want in g["values"].items():
        assert round(100 * diagnose.rmse_reduction(int(d), g["q"], g["r2"])) == want


def test_v_a_closed_form_against_integration():
    # E[chi2_d | chi2_d <= c] / d by quadrature of the density, independent of the
    # Pr(chi2_{d+2} <= c) identity in the Appendix A footnote.
    for d in [3, 30, 100]:
        c = diagnose.c_q(0.05, d)
        num, _ = integrate.quad(lambda x: x * stats.chi2.pdf(x, d), 0, c)
        den, _ = integrate.quad(lambda x: stats.chi2.pdf(x, d), 0, c)
        assert abs(num / den / d - diagnose.v_a(d, 0.05)) < 1e-7


def test_truncated_mean_monte_carlo():
    rng = np.random.default_rng(0)
    d, q = 10, 0.2
    z = rng.chisquare(d, size=400000)
    c = diagnose.c_q(q, d)
    assert abs(z[z <= c].mean() - diagnose.expected_M_accept(d, q)) < 0.02


def test_mse_forms():
    # E[MSE | accept] at q = 1 equals the complete-randomization MSE (v_a -> 1)
    a = diagnose.mse_accept(1.3, 0.4, 20, 1.0 - 1e-12, 50, 70)
    b = diagnose.mse_complete(1.3, 0.4, 50, 70)
    assert abs(a - b) / b < 1e-6
    # typical orientation never exceeds the Cauchy-Schwarz bound
    assert diagnose.rmse_typical(1, 0.5, 10, 0.3, 50, 50) <= diagnose.rmse_bound(1, 0.5, 0.3, 50, 50)


def _whitened_sample(n, d, seed):
    """Covariates whose sample covariance (denominator n - 1) is exactly I_d."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, d))
    Zc = Z - Z.mean(axis=0)
    L = np.linalg.cholesky(Zc.T @ Zc / (n - 1))
    return np.linalg.solve(L, Zc.T).T


def _dim(w, y):
    """Difference in means of y (last axis units) under the 0/1 vector w."""
    w = np.asarray(w, dtype=bool)
    return y[..., w].mean(axis=-1) - y[..., ~w].mean(axis=-1)


def _realised_case():
    n, n1, d = 60, 25, 5
    X = _whitened_sample(n, d, 11)
    w = np.zeros(n, dtype=np.uint8)
    w[np.random.default_rng(12).permutation(n)[:n1]] = 1
    M = balance.mahalanobis_batch(X, w[None, :], prep.prepare(X, n1)["S_lam"])[0]   # chi^2 scale
    M_paper = (1.0 / n1 + 1.0 / (n - n1)) * M
    return X, w, n1, n - n1, d, M_paper


def test_rmse_bound_reached_by_aligned_prognostic_direction():
    """Appendix A part A (Bound): with beta parallel to the realised imbalance Delta the squared
    bias (beta^T Delta)^2 equals sigma_prog^2 M, and the conditional MSE of the difference in
    means -- the squared bias of the noise-free outcome X beta plus the noise variance, here
    estimated by Monte Carlo over the noise -- equals rmse_bound^2.  Both sides come from data:
    the bias is the difference in means of X beta, M the textbook statistic."""
    X, w, n1, n0, d, M_paper = _realised_case()
    sigma, r2 = 0.7, 0.6
    sp2 = r2 / (1 - r2) * sigma ** 2
    delta = X[w == 1].mean(axis=0) - X[w == 0].mean(axis=0)
    beta = np.sqrt(sp2) * delta / np.linalg.norm(delta)
    assert abs(np.var(X @ beta, ddof=1) - sp2) < 1e-12 * sp2           # sigma_prog^2 = Var(beta^T X_i)
    bias = _dim(w, X @ beta)
    assert abs(bias ** 2 - sp2 * M_paper) < 1e-10 * sp2 * M_paper       # Cauchy-Schwarz with equality
    rng = np.random.default_rng(13)
    eps = rng.normal(0.0, sigma, size=(200_000, len(w)))
    err = bias + _dim(w, eps)                                           # tau_hat - tau
    mse = np.mean(err ** 2)
    bound = diagnose.rmse_bound(sigma, r2, M_paper, n1, n0) ** 2
    assert abs(mse - bound) < 4 * np.std(err ** 2) / np.sqrt(len(err)), (mse, bound)
    # a prognostic direction orthogonal to Delta leaves only the noise variance, below the bound
    b2 = np.linalg.svd(delta[None, :])[2][1]
    bias2 = _dim(w, X @ (np.sqrt(sp2) * b2))
    assert abs(bias2) < 1e-12 and sigma ** 2 * (1.0 / n1 + 1.0 / n0) < bound


def test_rmse_typical_is_the_orientation_average():
    """Appendix A part A (Typical orientation): averaged over prognostic directions uniform on the
    sphere at fixed ||beta||^2 = sigma_prog^2, the squared bias of the realised assignment is
    sigma_prog^2 M / d.  Monte Carlo over 200000 directions, bias from the data."""
    X, w, n1, n0, d, M_paper = _realised_case()
    sigma, r2 = 1.3, 0.45
    sp2 = r2 / (1 - r2) * sigma ** 2
    U = np.random.default_rng(14).standard_normal((200_000, d))
    B = np.sqrt(sp2) * U / np.linalg.norm(U, axis=1, keepdims=True)
    bias2 = _dim(w, B @ X.T) ** 2
    want = diagnose.rmse_typical(sigma, r2, d, M_paper, n1, n0) ** 2 - sigma ** 2 * (1.0 / n1 + 1.0 / n0)
    assert abs(bias2.mean() - want) < 4 * bias2.std() / np.sqrt(len(bias2)), (bias2.mean(), want)
    # d times the typical squared bias is the Cauchy-Schwarz worst case
    bound = diagnose.rmse_bound(sigma, r2, M_paper, n1, n0) ** 2 - sigma ** 2 * (1.0 / n1 + 1.0 / n0)
    assert abs(d * want - bound) < 1e-12 * bound


def _complete_randomization_errors(n, n1, d, sigma, r2, reps, seed, accept_c=None):
    """tau_hat - tau over (X, w, eps) drawn afresh: X rows iid N(0, I_d) (so Var(beta^T X_i) =
    ||beta||^2), w complete randomization, eps iid N(0, sigma^2); beta fixed.  With accept_c,
    only draws whose population-whitened imbalance ||Delta||^2 / (1/n1 + 1/n0) is <= accept_c
    are kept."""
    rng = np.random.default_rng(seed)
    sp2 = r2 / (1 - r2) * sigma ** 2
    beta = rng.standard_normal(d)
    beta *= np.sqrt(sp2) / np.linalg.norm(beta)
    X = rng.standard_normal((reps, n, d))
    W = np.argsort(rng.random((reps, n)), axis=1) < n1
    eps = rng.normal(0.0, sigma, size=(reps, n))
    Y = X @ beta + eps                                                  # tau w cancels in tau_hat - tau
    err = (np.where(W, Y, 0).sum(1) / n1) - (np.where(~W, Y, 0).sum(1) / (n - n1))
    if accept_c is not None:
        D = (np.where(W[:, :, None], X, 0).sum(1) / n1) - (np.where(~W[:, :, None], X, 0).sum(1) / (n - n1))
        keep = (D ** 2).sum(1) / (1.0 / n1 + 1.0 / (n - n1)) <= accept_c
        err = err[keep]
    return err


def test_mse_complete_monte_carlo():
    """Appendix A part B: E[MSE] = (1/n_T + 1/n_C)(sigma^2 + sigma_prog^2) under complete
    randomization, by Monte Carlo over covariates, assignment and noise."""
    n, n1, d, sigma, r2 = 30, 12, 4, 0.9, 0.5
    err = _complete_randomization_errors(n, n1, d, sigma, r2, 60_000, 21)
    mse = np.mean(err ** 2)
    want = diagnose.mse_complete(sigma, r2, n1, n - n1)
    assert abs(mse - want) < 4 * np.std(err ** 2) / np.sqrt(len(err)), (mse, want)


def test_mse_accept_monte_carlo():
    """Section 2.2 / Appendix A part C: E[MSE | M <= a] = (1/n_T + 1/n_C)(sigma^2 + v_a(d)
    sigma_prog^2); Gaussian covariates make the chi-square law of the whitened imbalance exact."""
    n, n1, d, sigma, r2, q = 30, 12, 4, 0.9, 0.6, 0.2
    err = _complete_randomization_errors(n, n1, d, sigma, r2, 150_000, 22, accept_c=diagnose.c_q(q, d))
    assert abs(len(err) / 150_000 - q) < 0.01
    mse = np.mean(err ** 2)
    want = diagnose.mse_accept(sigma, r2, d, q, n1, n - n1)
    assert abs(mse - want) < 4 * np.std(err ** 2) / np.sqrt(len(err)), (mse, want)
    assert want < diagnose.mse_complete(sigma, r2, n1, n - n1) * 0.85


def test_q_star_example_parity_unpinned(golden):
    """Parity unpinned: the printed q* ~ 1.2e-5 does not follow from Appendix A part D.

    The target needs RMSE^2 <= 0.2^2 / (1.96 + 0.84)^2 ~ 0.0051, i.e. v_a(1000) <= 0.41,
    while v_a(1000) at q = 1.2e-5 is about 0.81.  The test records that reading."""
    g = golden["q_star_example"]
    assert 0.80 < diagnose.v_a(g["d"], g["q_star"]) < 0.83
    assert diagnose.q_star(g["d"], g["n_t"], g["n_c"], g["sigma"], g["r2"], g["tau"],
                           g["alpha"], g["power"], q_lo=1e-30) is None
    # an easier target is met and the search returns its boundary
    qs = diagnose.q_star(30, 500, 500, 1.0, 0.5, 0.2)
    assert qs is not None and 0 < qs < 1
    target = 0.2 ** 2 / (stats.norm.ppf(0.975) + stats.norm.ppf(0.8)) ** 2
    assert abs(diagnose.mse_accept(1.0, 0.5, 30, qs, 500, 500) - target) < 1e-9


def test_key_memory_factor(golden):
    g = golden["key_memory"]
    assert g["n"] / g["L"] == g["factor"]
