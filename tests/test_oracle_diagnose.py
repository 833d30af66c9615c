"""Pins for the design closed forms against the paper's printed numbers (CPU only)."""

import numpy as np
from scipy import integrate, stats

from oracle import diagnose


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
