// Design diagnostics: closed forms for choosing the acceptance stringency (section 2.2;
// Appendix A parts A-D).  Host code, double precision.
//
// Under complete randomization with whitened covariates, M (chi^2 scale) is approximately
// chi^2_d.  Accepting M <= c_q, c_q the q-quantile of chi^2_d, shrinks the variance of each
// whitened covariate's difference in means by v_a(d) = Pr(chi^2_{d+2} <= c_q) /
// Pr(chi^2_d <= c_q) (Appendix A part C), so the conditional MSE of the difference in
// means is (1/n1 + 1/n0)(sigma^2 + v_a sigma_prog^2) with sigma_prog^2 = R^2/(1-R^2) sigma^2
// (section 2.2; Appendix A part B).  q* is the largest q meeting an RMSE target derived from
// a power requirement (Appendix A part D).
//
// Numerics (written from the definitions): the regularised lower incomplete gamma P(a, x)
// by its power series for x < a + 1 and by the continued fraction of Q = 1 - P (modified
// Lentz evaluation) otherwise; chi^2_d CDF F(x) = P(d/2, x/2); quantiles by safeguarded
// Newton steps on log F inside a bisection bracket; v_a from the recurrence
// P(a + 1, x) = P(a, x) - x^a e^-x / Gamma(a + 1), which stays accurate when both
// probabilities are tiny; normal quantiles by Newton on erfc.
#include <cmath>
#include <limits>

#include "rr_internal.h"

namespace rr {
namespace {

// Series: P(a, x) = x^a e^-x / Gamma(a + 1) * (1 + rest), rest = sum_{k>=1} x^k / ((a+1)...(a+k)),
// for x < a + 1; the tail is kept apart from the leading 1 so that tiny tails stay exact.
double p_series_rest(double a, double x) {
    double term = 1.0, rest = 0.0;
    for (int k = 1; k < 100000; ++k) {
        term *= x / (a + k);
        rest += term;
        if (term < (1.0 + rest) * 1e-17) break;
    }
    return rest;
}

double log_p_series(double a, double x) {
    return a * std::log(x) - x - std::lgamma(a + 1.0) + std::log1p(p_series_rest(a, x));
}

// Q(a, x) by the continued fraction x^a e^-x / Gamma(a) * 1/(x + 1 - a - 1(1-a)/(x + 3 - a - ...))
double q_cfrac(double a, double x) {
    const double tiny = 1e-300;
    double b = x + 1.0 - a, c = 1.0 / tiny, d = 1.0 / b, h = d;
    for (int i = 1; i < 100000; ++i) {
        const double an = -i * (i - a);
        b += 2.0;
        d = an * d + b;
        if (std::fabs(d) < tiny) d = tiny;
        c = b + an / c;
        if (std::fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        const double del = d * c;
        h *= del;
        if (std::fabs(del - 1.0) < 1e-16) break;
    }
    return std::exp(a * std::log(x) - x - std::lgamma(a)) * h;
}

// log P(a, x), x >= 0
double log_gamma_p(double a, double x) {
    if (x <= 0.0) return -std::numeric_limits<double>::infinity();
    if (x < a + 1.0) return log_p_series(a, x);
    return std::log1p(-q_cfrac(a, x));
}

double chi2_log_cdf(double x, double d) { return log_gamma_p(0.5 * d, 0.5 * x); }

// x with F_{chi^2_d}(x) = q, 0 < q < 1
double chi2_quantile(double q, double d) {
    const double lq = std::log(q);
    double lo = 0.0, hi = std::max(1.0, d);
    while (chi2_log_cdf(hi, d) < lq) hi *= 2.0;
    double x = 0.5 * (lo + hi);
    for (int it = 0; it < 400; ++it) {
        const double f = chi2_log_cdf(x, d) - lq;
        if (f < 0) lo = x; else hi = x;
        // Newton on log F: d/dx log F = pdf / F
        const double lpdf = (0.5 * d - 1.0) * std::log(x) - 0.5 * x - 0.5 * d * std::log(2.0) - std::lgamma(0.5 * d);
        const double slope = std::exp(lpdf - chi2_log_cdf(x, d));
        double nx = x - f / slope;
        if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
        if (std::fabs(nx - x) <= 1e-15 * x || hi - lo <= 1e-15 * hi) {
            x = nx;
            break;
        }
        x = nx;
    }
    return x;
}

// Pr(chi^2_{d+2} <= c) / Pr(chi^2_d <= c) = 1 - (c/2)^{d/2} e^{-c/2} / (Gamma(d/2 + 1) P(d/2, c/2))
// (in the series regime the ratio is rest / (1 + rest) exactly)
double v_a_of(double c, double d) {
    const double a = 0.5 * d, x = 0.5 * c;
    if (x < a + 1.0) {
        const double rest = p_series_rest(a, x);
        return rest / (1.0 + rest);
    }
    const double lnum = a * std::log(x) - x - std::lgamma(a + 1.0);
    return -std::expm1(lnum - log_gamma_p(a, x));
}

double normal_quantile(double p) {
    // Newton on Phi(z) = erfc(-z / sqrt 2) / 2 from a bisection bracket
    double lo = -40.0, hi = 40.0, z = 0.0;
    for (int it = 0; it < 200; ++it) {
        const double f = 0.5 * std::erfc(-z / std::sqrt(2.0)) - p;
        if (f < 0) lo = z; else hi = z;
        const double pdf = std::exp(-0.5 * z * z) / std::sqrt(2.0 * M_PI);
        double nz = pdf > 0 ? z - f / pdf : 0.5 * (lo + hi);
        if (!(nz > lo && nz < hi)) nz = 0.5 * (lo + hi);
        if (std::fabs(nz - z) < 1e-15 * (1.0 + std::fabs(z))) return nz;
        z = nz;
    }
    return z;
}

bool valid_design(int64_t n1, int64_t n0, int64_t d, double sigma, double r2) {
    return n1 >= 1 && n0 >= 1 && d >= 1 && sigma > 0 && std::isfinite(sigma) && r2 >= 0 && r2 < 1;
}

double mse_accept_of(double v, double sigma, double r2, double sc) {
    return sc * (sigma * sigma + v * r2 / (1.0 - r2) * sigma * sigma);
}

}  // namespace

double chi2_quantile_of(double q, double d) { return q >= 1.0 ? INFINITY : chi2_quantile(q, d); }

}  // namespace rr

using namespace rr;

extern "C" rr_status rr_diagnose(int64_t n1, int64_t n0, int64_t d, double q, double sigma, double r2,
                                 rr_design* out) {
    if (!out || !valid_design(n1, n0, d, sigma, r2) || !(q > 0.0 && q <= 1.0)) {
        set_error("rr_diagnose: invalid argument");
        return RR_E_ARG;
    }
    const double dd = (double)d, sc = 1.0 / (double)n1 + 1.0 / (double)n0;
    rr_design r{};
    if (q >= 1.0) {
        r.c_q = INFINITY;
        r.v_a = 1.0;
    } else {
        r.c_q = chi2_quantile(q, dd);
        r.v_a = v_a_of(r.c_q, dd);
    }
    r.a_q = sc * r.c_q;
    r.expected_M = dd * r.v_a;
    const double sp = r2 / (1.0 - r2);
    r.rmse_reduction = 1.0 - std::sqrt((1.0 + r.v_a * sp) / (1.0 + sp));
    r.mse_complete = sc * (sigma * sigma + sp * sigma * sigma);
    r.mse_accept = mse_accept_of(r.v_a, sigma, r2, sc);
    *out = r;
    return RR_OK;
}

extern "C" rr_status rr_q_star(int64_t n1, int64_t n0, int64_t d, double sigma, double r2, double tau,
                               double alpha, double power, double q_lo, double* q_star) {
    if (!q_star || !valid_design(n1, n0, d, sigma, r2) || !(tau != 0.0 && std::isfinite(tau)) ||
        !(alpha > 0.0 && alpha < 1.0) || !(power > 0.0 && power < 1.0) || !(q_lo > 0.0 && q_lo < 1.0)) {
        set_error("rr_q_star: invalid argument");
        return RR_E_ARG;
    }
    const double dd = (double)d, sc = 1.0 / (double)n1 + 1.0 / (double)n0;
    const double z = normal_quantile(1.0 - 0.5 * alpha) + normal_quantile(power);
    const double target = tau * tau / (z * z);
    auto gap = [&](double lq) {
        const double q = std::exp(lq);
        const double v = q >= 1.0 ? 1.0 : v_a_of(chi2_quantile(q, dd), dd);
        return mse_accept_of(v, sigma, r2, sc) - target;
    };
    if (gap(0.0) <= 0.0) {
        *q_star = 1.0;
        return RR_OK;
    }
    double lo = std::log(q_lo), hi = 0.0;
    if (gap(lo) > 0.0) {
        set_error("rr_q_star: the RMSE target is not met for any q >= q_lo");
        return RR_E_RANGE;
    }
    // v_a increases with q: the feasible set is (0, q*]; bisect on log q
    for (int it = 0; it < 200 && hi - lo > 1e-13 * (1.0 + std::fabs(lo)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (gap(mid) <= 0.0) lo = mid; else hi = mid;
    }
    *q_star = std::exp(lo);
    return RR_OK;
}

extern "C" rr_status rr_realized_rmse(int64_t n1, int64_t n0, int64_t d, double M, double sigma, double r2,
                                      double* rmse_typical, double* rmse_bound) {
    if (!rmse_typical || !rmse_bound || !valid_design(n1, n0, d, sigma, r2) || !(M >= 0.0) || !std::isfinite(M)) {
        set_error("rr_realized_rmse: invalid argument");
        return RR_E_ARG;
    }
    // the realised imbalance on the paper's scale, ||Delta||^2 = (1/n1 + 1/n0) M
    const double sc = 1.0 / (double)n1 + 1.0 / (double)n0;
    const double m_paper = sc * M;
    const double noise = sigma * sigma * sc;                      // irreducible residual variance
    const double prog = r2 / (1.0 - r2) * sigma * sigma;         // sigma_prog^2
    *rmse_typical = std::sqrt(noise + prog / (double)d * m_paper);
    *rmse_bound = std::sqrt(noise + prog * m_paper);
    return RR_OK;
}
