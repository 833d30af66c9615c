"""Library design diagnostics (host code in librr) vs the oracle's SciPy closed forms and the
paper's printed numbers.  CPU only: these calls do no device work."""

import math

import numpy as np
import pytest

from oracle import diagnose


@pytest.fixture(scope="module")
def rr():
    import paper_2501_07642_amd as rr
    try:
        rr.load()
    except (OSError, RuntimeError) as e:
        pytest.skip(f"librr.so not loadable here: {e}")
    return rr


DS = [1, 2, 3, 10, 30, 100, 500, 1000, 5000]
QS = [1e-12, 1.2e-5, 1e-3, 0.01, 0.1, 0.5, 0.9, 0.999]


def test_quantile_and_shrinkage_match_scipy(rr):
    for d in DS:
        for q in QS:
            r = rr.rr_diagnose(50, 70, d, q, 1.0, 0.3)
            c = diagnose.c_q(q, d)
            assert abs(r["c_q"] - c) <= 1e-10 * c, (d, q, r["c_q"], c)
            v = diagnose.v_a(d, c=c)
            assert abs(r["v_a"] - v) <= 1e-9 * v, (d, q, r["v_a"], v)
            assert abs(r["a_q"] - diagnose.a_q(q, d, 50, 70)) <= 1e-10 * r["a_q"]
            assert abs(r["expected_M"] - d * v) <= 1e-9 * d * v
            assert abs(r["mse_accept"] - diagnose.mse_accept(1.0, 0.3, d, q, 50, 70)) <= 1e-9 * r["mse_accept"]
            assert abs(r["rmse_reduction"] - diagnose.rmse_reduction(d, q, 0.3)) <= 1e-9


def test_paper_numbers(rr, golden):
    g = golden["v_a_q001"]
    for d, want in g["values"].items():
        assert round(rr.rr_diagnose(100, 100, int(d), g["q"])["v_a"], g["decimals"]) == want
    g = golden["rmse_drop_pct"]
    for d, want in g["values"].items():
        assert round(100 * rr.rr_diagnose(100, 100, int(d), g["q"], 1.0, g["r2"])["rmse_reduction"]) == want


def test_special_cases(rr):
    # q = 1: no rerandomization, v_a = 1 and the conditional MSE is the complete one
    r = rr.rr_diagnose(10, 30, 7, 1.0, 2.0, 0.5)
    assert math.isinf(r["c_q"]) and r["v_a"] == 1.0
    assert abs(r["mse_accept"] - diagnose.mse_complete(2.0, 0.5, 10, 30)) <= 1e-12 * r["mse_accept"]
    # d = 2: chi^2_2 is exponential with mean 2, so c_q = -2 log(1 - q) in closed form
    for q in [1e-9, 0.01, 0.3]:
        assert abs(rr.rr_diagnose(5, 5, 2, q)["c_q"] + 2 * math.log1p(-q)) <= 1e-12 * rr.rr_diagnose(5, 5, 2, q)["c_q"]
    # v_a decreases as q shrinks and lies in (0, 1)
    vs = [rr.rr_diagnose(50, 50, 20, q)["v_a"] for q in [1e-8, 1e-4, 1e-2, 0.5]]
    assert all(0 < v < 1 for v in vs) and np.all(np.diff(vs) > 0)


def test_q_star(rr, golden):
    g = golden["q_star_example"]
    assert rr.rr_q_star(g["n_t"], g["n_c"], g["d"], g["sigma"], g["r2"], g["tau"], g["alpha"], g["power"],
                        1e-30) is None
    qs = rr.rr_q_star(500, 500, 30, 1.0, 0.5, 0.2)
    want = diagnose.q_star(30, 500, 500, 1.0, 0.5, 0.2)
    assert abs(qs - want) <= 1e-6 * want
    # an easy target is met without rerandomization
    assert rr.rr_q_star(500, 500, 30, 1.0, 0.5, 5.0) == 1.0


def test_errors(rr):
    for args in [(0, 5, 3, 0.1), (5, 5, 0, 0.1), (5, 5, 3, 0.0), (5, 5, 3, 1.5)]:
        with pytest.raises(rr.RRError) as e:
            rr.rr_diagnose(*args)
        assert e.value.status == "RR_E_ARG"
    with pytest.raises(rr.RRError):
        rr.rr_diagnose(5, 5, 3, 0.1, 1.0, 1.0)
    with pytest.raises(rr.RRError):
        rr.rr_q_star(5, 5, 3, 1.0, 0.5, 0.0)


def test_realized_rmse_matches_oracle(rr):
    """Appendix A part A: typical-orientation RMSE and Cauchy-Schwarz bound of a realised M
    (library on the chi^2 scale, oracle on the paper's scale (1/n1 + 1/n0) M)."""
    for n1, n0, d, M, sigma, r2 in [(500, 500, 1000, 866.0, 1.0, 0.4), (10, 30, 3, 0.05, 2.0, 0.9),
                                    (50, 70, 20, 0.0, 0.5, 0.0), (7, 7, 1, 3.2, 1.0, 0.5)]:
        t, b = rr.rr_realized_rmse(n1, n0, d, M, sigma, r2)
        mp = (1.0 / n1 + 1.0 / n0) * M
        assert abs(t - diagnose.rmse_typical(sigma, r2, d, mp, n1, n0)) <= 1e-13 * t
        assert abs(b - diagnose.rmse_bound(sigma, r2, mp, n1, n0)) <= 1e-13 * b
        assert t <= b
    # at d = 1 the typical orientation is the bound (one direction only)
    t, b = rr.rr_realized_rmse(7, 9, 1, 2.5, 1.0, 0.3)
    assert abs(t - b) <= 1e-15 * b
    for args in [(5, 5, 3, -1.0), (5, 5, 3, float("nan")), (0, 5, 3, 1.0)]:
        with pytest.raises(rr.RRError):
            rr.rr_realized_rmse(*args)
