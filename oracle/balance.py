"""The Mahalanobis balance statistic, textbook form.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 2.2 defines the imbalance of a realised assignment through the treated-minus-
control mean difference Delta = xbar_T - xbar_C of whitened covariates, M = Delta^T Delta;
the Appendix A remark on general Sigma_X writes it as Delta^T Sigma_X^-1 Delta.  Under
complete randomization Delta has covariance (1/n_T + 1/n_C) Sigma_X, and section 2.2
states M ~ (1/n_T + 1/n_C) chi^2_d.  This build reports M on the chi^2_d scale:

    M(w) = (n1 * n0 / n) * Delta^T S_lam^-1 Delta,

i.e. the paper's M divided by (1/n1 + 1/n0) = n / (n1 n0).  The oracle evaluates it
literally: group means of the raw covariates, their difference, a linear solve with the
(ridged) covariance.  It deliberately does not use the centred/whitened sum that the GPU
path contracts, so that the two algebras check each other.

A second criterion, ``max_smd_batch``, scores an assignment by its worst single covariate
instead of the sum over covariates: section 2.2 writes M as the sum of the squared
standardised mean differences SMD_j of the columns; the per-column criterion takes the largest
of them, on the same chi^2 scale (each term is chi^2_1 under complete randomization):

    M_max(w) = (n1 * n0 / n) * max_j Delta_j^2 / (S_jj + lambda).
"""

import numpy as np


def mahalanobis_batch(X, W, S_lam):
    """M for every row of a 0/1 matrix W (B x n) with a common n1."""
    X = np.asarray(X, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    n = X.shape[0]
    n1 = W[0].sum()
    n0 = n - n1
    xbar_t = W @ X / n1
    xbar_c = (1.0 - W) @ X / n0
    delta = xbar_t - xbar_c                       # B x d
    sol = np.linalg.solve(S_lam, delta.T).T       # B x d
    return n1 * n0 / n * np.einsum("bj,bj->b", delta, sol)


def max_smd_batch(X, W, var):
    """M_max for every row of a 0/1 matrix W (B x n): the largest squared standardised mean
    difference, (n1 n0 / n) max_j Delta_j^2 / var_j, var_j the (ridged) column variance."""
    X = np.asarray(X, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    var = np.asarray(var, dtype=np.float64)
    n = X.shape[0]
    n1 = W[0].sum()
    n0 = n - n1
    delta = W @ X / n1 - (1.0 - W) @ X / n0      # B x d
    return n1 * n0 / n * np.max(delta * delta / var, axis=1)
