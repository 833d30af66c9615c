"""Seeded synthetic inputs shared by the HIP path's tests, the benchmark and the oracle.

This module holds data generation only -- covariates, outcomes, null grids and the
workload table -- and none of the method's arithmetic.  The paper benchmarks on
unspecified controlled synthetic data (section 4, "Impact"); the shapes here follow its
benchmark grid (n = 100 / 1000, d up to 1000, q down to 0.00025), its usage snippet
(Appendix B: n = 200, n1 = 100, d = 50, q = 0.01, 2e5 draws, batches of 1e4, tau = 1,
noise sd 0.5) and its motivating example (about 1000 units, 768 embedding features,
section 3).
"""

import numpy as np


def gaussian_X(n, d, seed, dtype=np.float64):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, d)).astype(dtype)


def ar1_t_X(n, d, seed, rho=0.5, t_cols=100, t_df=5):
    """Columns 0..d-t_cols-1: AR(1) across columns with correlation rho (Gaussian);
    the last t_cols columns: iid Student-t(t_df), unscaled."""
    rng = np.random.default_rng(seed)
    X = np.empty((n, d), dtype=np.float64)
    g = d - t_cols
    z = rng.standard_normal((n, g))
    X[:, 0] = z[:, 0]
    c = np.sqrt(1.0 - rho * rho)
    for j in range(1, g):
        X[:, j] = rho * X[:, j - 1] + c * z[:, j]
    X[:, g:] = rng.standard_t(t_df, size=(n, t_cols))
    return X


def outcomes(X, w_obs, tau, noise_sd, seed):
    """Y = X beta + tau * w_obs + N(0, noise_sd^2), beta ~ N(0, I)."""
    rng = np.random.default_rng(seed)
    X = np.asarray(X, dtype=np.float64)
    beta = rng.standard_normal(X.shape[1])
    eps = rng.normal(0.0, noise_sd, size=X.shape[0])
    return X @ beta + tau * np.asarray(w_obs, dtype=np.float64) + eps


def tau_grid(lo=-2.0, hi=2.0, num=201):
    return np.linspace(lo, hi, num)


def batched_shapes(num_problems, seed, n_range=(50, 2000), d_range=(10, 500)):
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=num_problems)
    ds = rng.integers(d_range[0], d_range[1] + 1, size=num_problems)
    return [(int(n), int(n) // 2, int(d)) for n, d in zip(ns, ds)]


# The five workloads.  Seeds are fixed here so that every consumer sees the same data.
WORKLOADS = {
    "exact_n20_d3": dict(
        kind="exact", n=20, n1=10, d=3, x="gaussian", x_seed=101, ridge_rel=0.0,
        mode="quantile", q=0.01, tau=1.0, noise_sd=1.0, y_seed=102,
        taus=[0.0] + list(np.linspace(-3.0, 3.0, 25)), obs_seed=103),
    "mc_n100_d100": dict(
        kind="mc", n=100, n1=50, d=100, x="gaussian", x_seed=201, ridge_rel=1e-2,
        seed=0x5EED0002, key_begin=0, num_draws=200_000, mode="quantile", q=0.01,
        precision="fp32", tau=0.5, noise_sd=1.0, y_seed=202,
        taus=list(np.linspace(-2.0, 2.0, 201)), obs_seed=203),
    "precision_n1000_d1000": dict(
        kind="mc", n=1000, n1=500, d=1000, x="ar1_t", x_seed=301, ridge_rel=1e-2,
        seed=0x5EED0003, key_begin=0, num_draws=200_000, mode="quantile", q=0.01,
        precision="split_bf16", tau=0.5, noise_sd=1.0, y_seed=302,
        taus=list(np.linspace(-2.0, 2.0, 201)), obs_seed=303),
    "stream_n1000_d1000": dict(
        kind="mc", n=1000, n1=500, d=1000, x="gaussian", x_seed=401, ridge_rel=1e-2,
        seed=0x5EED0004, key_begin=0, num_draws=100_000_000, mode="quantile", q=1.2e-5,
        precision="split_bf16", tau=0.5, noise_sd=1.0, y_seed=402,
        taus=list(np.linspace(-2.0, 2.0, 201)), obs_seed=403),
    "highdim_n256_d768": dict(
        kind="mc", n=256, n1=128, d=768, x="gaussian", x_seed=601, ridge_rel=0.0, metric="diagonal",
        seed=0x5EED0006, key_begin=0, num_draws=100_000_000, mode="quantile", q=1e-4,
        precision="gram_bf16", tau=0.5, noise_sd=1.0, y_seed=602,
        taus=list(np.linspace(-2.0, 2.0, 201)), obs_seed=603),
    # a small streaming pool of more than 16 chunks of 2^20 draws whose keys cross 2^32: the
    # running acceptance bound is refreshed twice while streaming (a parity case, not a bench line)
    "refresh_n64_d8": dict(
        kind="mc", n=64, n1=32, d=8, x="gaussian", x_seed=701, ridge_rel=0.0,
        seed=0x5EED0007, key_begin=(1 << 32) - 3_000_000, num_draws=16 * (1 << 20) + (1 << 19) + 77,
        mode="quantile", q=1e-4, precision="split_bf16", tau=0.5, noise_sd=1.0, y_seed=702,
        taus=list(np.linspace(-2.0, 2.0, 21)), obs_seed=703),
    "batched_512": dict(
        kind="batched", num_problems=512, shape_seed=501, x_seed_base=10_000,
        ridge_rel=1e-2, seed_base=0x5EED0500, key_begin=0, num_draws=100_000,
        mode="quantile", q=0.01, precision="split_bf16"),
}


def workload_X(name):
    w = WORKLOADS[name]
    if w["x"] == "gaussian":
        return gaussian_X(w["n"], w["d"], w["x_seed"])
    if w["x"] == "ar1_t":
        return ar1_t_X(w["n"], w["d"], w["x_seed"])
    raise KeyError(w["x"])


def batched_problem(p, workload="batched_512"):
    """(X float32, n1, seed) of problem p of the batched workload."""
    w = WORKLOADS[workload]
    n, n1, d = batched_shapes(w["num_problems"], w["shape_seed"])[p]
    X = gaussian_X(n, d, w["x_seed_base"] + p, dtype=np.float32)
    return X, n1, w["seed_base"] + p


def obs_pick(num_accepted, seed):
    """Index of the observed assignment among the accepted keys (sorted ascending)."""
    return int(np.random.default_rng(seed).integers(0, num_accepted))
