"""Covariance, ridge and feasibility of the whitening step.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 2.2 assumes covariates whitened so that Sigma_X is the identity, and the
Appendix A remark on general Sigma_X reduces M = Delta^T Sigma_X^-1 Delta to the
whitened case.  The readings implemented here:

* Sigma_X is the sample covariance over all n units, with denominator n - 1, fixed for
  every candidate draw (the default metric is called Hotelling's T^2 in section 2.3;
  a per-draw pooled covariance would change with the draw).
* A ridge lambda = ridge_rel * tr(S) / d is added to the diagonal.  With ridge_rel = 0,
  a covariance whose Cholesky factorisation fails, or whose smallest squared pivot is
  below 1e-10 times the largest diagonal entry of S, is reported as singular.  The paper
  passes an undefined ``approximate_inv = TRUE`` in its usage snippet (Appendix B); the
  ridge is this build's reading of it for d >= n - 1.
* metric = "diagonal": the covariates are standardised but not decorrelated, i.e.
  S_lam is replaced by its diagonal, so M sums squared standardised mean differences
  (section 2.2 writes M for standardised covariates; a diagonal approximation is also one
  reading of ``approximate_inv``).  A variance below 1e-10 times the largest one is
  reported as singular.
* metric = "max_smd": the same standardisation, for the per-column criterion (the largest
  squared standardised mean difference instead of their sum, see ``balance``).
"""

import numpy as np

SINGULAR_RATIO = 1e-10


class SingularCovariance(ValueError):
    pass


def covariance(X):
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    mu = X.mean(axis=0)
    Xc = X - mu
    return mu, Xc.T @ Xc / (n - 1)


def prepare(X, n1, ridge_rel=0.0, metric="mahalanobis"):
    """Return dict(mu, S, lam, S_lam, L) for covariates X (n x d)."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    if not (1 <= n1 <= n - 1) or d < 1 or ridge_rel < 0 or metric not in ("mahalanobis", "diagonal", "max_smd"):
        raise ValueError("bad arguments")
    mu, S = covariance(X)
    lam = ridge_rel * np.trace(S) / d
    S_lam = S + lam * np.eye(d)
    if metric in ("diagonal", "max_smd"):
        S_lam = np.diag(np.diag(S_lam))
    try:
        L = np.linalg.cholesky(S_lam)
    except np.linalg.LinAlgError as e:
        raise SingularCovariance(str(e)) from e
    if np.min(np.diag(L)) ** 2 < SINGULAR_RATIO * np.max(np.diag(S)):
        raise SingularCovariance("pivot below threshold")
    return dict(mu=mu, S=S, lam=lam, S_lam=S_lam, L=L, n=n, d=d, n1=n1, metric=metric)
