"""Closed forms for choosing stringency (section 2.2; Appendix A parts A-D).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  SciPy's chi-square distribution is
used as the library primitive.  n_T, n_C are the group sizes; M_paper denotes the
statistic on the paper's scale, M_paper = (1/n_T + 1/n_C) * M with M on the chi^2_d
scale that the library reports.
"""

import math

from scipy import optimize, stats


def scale(n_t, n_c):
    return 1.0 / n_t + 1.0 / n_c


def c_q(q, d):
    """c_q = F^-1_{chi^2_d}(q) (section 2.2)."""
    return float(stats.chi2.ppf(q, d))


def a_q(q, d, n_t, n_c):
    """Threshold on the paper's scale, a_q = (1/n_T + 1/n_C) c_q (section 2.2)."""
    return scale(n_t, n_c) * c_q(q, d)


def v_a(d, q=None, c=None):
    """Shrinkage factor v_a(d) = Pr(chi^2_{d+2} <= c) / Pr(chi^2_d <= c) (Appendix A part C)."""
    if c is None:
        c = c_q(q, d)
    return float(stats.chi2.cdf(c, d + 2) / stats.chi2.cdf(c, d))


def rmse_typical(sigma, r2, d, M_paper, n_t, n_c):
    """Typical-orientation RMSE of the difference in means (section 2.2, Appendix A part A)."""
    return math.sqrt(sigma ** 2 * scale(n_t, n_c) + r2 / (1 - r2) * sigma ** 2 / d * M_paper)


def rmse_bound(sigma, r2, M_paper, n_t, n_c):
    """Cauchy-Schwarz worst case: (beta^T Delta)^2 <= sigma_prog^2 M (Appendix A part A)."""
    return math.sqrt(sigma ** 2 * scale(n_t, n_c) + r2 / (1 - r2) * sigma ** 2 * M_paper)


def mse_complete(sigma, r2, n_t, n_c):
    """E[MSE] under complete randomization (Appendix A part B)."""
    return scale(n_t, n_c) * (sigma ** 2 + r2 / (1 - r2) * sigma ** 2)


def mse_accept(sigma, r2, d, q, n_t, n_c):
    """E[MSE | accept] = (1/n_T + 1/n_C)(sigma^2 + v_a(d) sigma_prog^2) (section 2.2, A part C)."""
    return scale(n_t, n_c) * (sigma ** 2 + v_a(d, q) * r2 / (1 - r2) * sigma ** 2)


def rmse_reduction(d, q, r2):
    """Relative RMSE drop of rerandomization at level q versus complete randomization."""
    sp = r2 / (1 - r2)
    return 1.0 - math.sqrt((1.0 + v_a(d, q) * sp) / (1.0 + sp))


def expected_M_accept(d, q):
    """E[M | M <= a] on the chi^2_d scale, d * v_a(d) (Appendix A part C, last display)."""
    return d * v_a(d, q)


def q_star(d, n_t, n_c, sigma, r2, tau, alpha=0.05, power=0.8, q_lo=1e-300):
    """Largest q with RMSE^2(q) <= tau^2 / (z_{1-alpha/2} + z_{power})^2 (Appendix A part D).

    Returns None when even q -> q_lo cannot meet the target.  v_a(d) increases with q, so
    the feasible set is an interval (0, q*]; a scalar root search finds its end.
    """
    target = tau ** 2 / (stats.norm.ppf(1 - alpha / 2) + stats.norm.ppf(power)) ** 2

    def gap(logq):
        return mse_accept(sigma, r2, d, math.exp(logq), n_t, n_c) - target

    if gap(0.0) <= 0:
        return 1.0
    lo = math.log(q_lo)
    if gap(lo) > 0:
        return None
    return math.exp(optimize.brentq(gap, lo, 0.0, xtol=1e-12))
