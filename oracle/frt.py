"""Randomization test conditioned on acceptance, with exact rational arithmetic.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 2.3 ("randomization_test()") and section 4 ("Design-based inference"): the
observed difference in means is compared with its distribution over the *accepted*
assignments only, giving a p-value for a sharp null that is bounded below by 1 / K
(K = number of accepted draws); inverting the test over a grid of nulls gives a fiducial
interval.  Readings implemented here:

* Sharp null H0(tau0): Y_i(1) - Y_i(0) = tau0 for every unit.  Under it the control
  outcomes are Y(0) = Y - tau0 * w_obs, and the statistic an accepted draw w_k would
  have produced is T_k(tau0) = DiM(w_k, Y - tau0 * w_obs); the observed one is
  T_obs(tau0) = DiM(w_obs, Y - tau0 * w_obs).  DiM(w, Z) = mean of Z over treated units
  minus mean over control units.
* p(tau0) = #{k : |T_k(tau0)| >= |T_obs(tau0)|} / K (two-sided, ties count as extreme).
  w_obs must be one of the accepted draws, as in the paper's usage snippet (Appendix B),
  so p >= 1 / K.
* Exactness: Y is first put on a fixed-point grid, Yq_i = rint(Y_i * 2^s) (round half
  to even), with s = 61 - t - e where n^2 <= 2^t and max|Y| = f * 2^e, f in [0.5, 1).
  All later arithmetic on Yq and on the (dyadic) tau0 values is exact.
* Interval: grid points with p > alpha (alpha = 0.05); reported as [min, max] of those
  points, with a flag when the accepted points are not contiguous on the grid.
"""

import math
from fractions import Fraction

import numpy as np

ALPHA = 0.05


def quantization_shift(Y, n):
    m = float(np.max(np.abs(np.asarray(Y, dtype=np.float64)))) if len(Y) else 0.0
    if m == 0.0:
        return 0
    _, e = math.frexp(m)
    t = (n * n - 1).bit_length()
    return 61 - t - e


def quantize(Y, s):
    """Yq_i = rint(Y_i * 2^s) as Python ints (float round() is round-half-even)."""
    return [int(round(math.ldexp(float(y), s))) for y in Y]


def dim_exact(w, Z):
    """Difference in means of the exact values Z (Fractions/ints) under 0/1 vector w."""
    w = np.asarray(w).astype(bool)
    zt = sum((Z[i] for i in np.nonzero(w)[0]), Fraction(0))
    zc = sum((Z[i] for i in np.nonzero(~w)[0]), Fraction(0))
    return zt / int(w.sum()) - zc / int((~w).sum())


def rand_test(W, obs, Y, taus):
    """Counts c_g, p-values, tau_hat and interval for accepted assignments W (K x n).

    ``obs`` is the row of W holding the observed assignment.  ``taus`` may hold floats
    or Fractions.  Per draw the treated sum of imputed control outcomes is split as
    sum_{i in T_k} (Yq_i - tau' w_obs,i) = A_k - tau' B_k with A_k the treated sum of Yq
    and B_k = |T_k and T_obs|, evaluated in exact integers / Fractions.
    """
    W = np.asarray(W, dtype=np.uint8)
    K, n = W.shape
    Y = np.asarray(Y, dtype=np.float64)
    s = quantization_shift(Y, n)
    Yq = quantize(Y, s)
    wo = W[obs].astype(np.int64)
    n1 = int(wo.sum())
    n0 = n - n1
    Yq_obj = np.array(Yq, dtype=object)
    A = [int(x) for x in W.astype(object) @ Yq_obj]          # exact treated sums
    B = [int(x) for x in W.astype(np.int64) @ wo]             # overlap with w_obs
    total = sum(Yq)
    counts = []
    for tau in taus:
        tq = Fraction(tau) * (Fraction(2) ** s)
        # sum of Z = Yq - tq * w_obs over all units
        zsum = total - tq * n1

        def dim(k):
            st = A[k] - tq * B[k]
            return st / n1 - (zsum - st) / n0

        t_obs = abs(dim(obs))
        counts.append(sum(1 for k in range(K) if abs(dim(k)) >= t_obs))
    tau_hat = Fraction(n * A[obs] - n1 * total, n1 * n0) / (Fraction(2) ** s)
    p = [c / K for c in counts]
    return dict(counts=counts, p=p, tau_hat=float(tau_hat), tau_hat_exact=tau_hat,
                shift=s, Yq=Yq, interval=interval(taus, p))


def rand_test_definition(W, obs, Y, taus):
    """Slow form: DiM of the imputed outcome vector per draw, straight from the definition."""
    W = np.asarray(W, dtype=np.uint8)
    K, n = W.shape
    s = quantization_shift(Y, n)
    Yq = quantize(Y, s)
    counts = []
    for tau in taus:
        tq = Fraction(tau) * (Fraction(2) ** s)
        Z = [Yq[i] - tq * int(W[obs, i]) for i in range(n)]
        t_obs = abs(dim_exact(W[obs], Z))
        counts.append(sum(1 for k in range(K) if abs(dim_exact(W[k], Z)) >= t_obs))
    return counts


def rand_test_unquantized(W, obs, Y, taus):
    """Same counts on the raw doubles (exact rationals), without the fixed-point grid."""
    W = np.asarray(W, dtype=np.uint8)
    K, n = W.shape
    counts = []
    for tau in taus:
        tf = Fraction(tau)
        Z = [Fraction(float(Y[i])) - tf * int(W[obs, i]) for i in range(n)]
        t_obs = abs(dim_exact(W[obs], Z))
        counts.append(sum(1 for k in range(K) if abs(dim_exact(W[k], Z)) >= t_obs))
    return counts


def interval(taus, p, alpha=ALPHA):
    taus = [float(t) for t in taus]
    keep = [i for i, pv in enumerate(p) if pv > alpha]
    if not keep:
        return dict(lo=None, hi=None, contiguous=True)
    contiguous = keep == list(range(keep[0], keep[-1] + 1))
    return dict(lo=min(taus[i] for i in keep), hi=max(taus[i] for i in keep),
                contiguous=contiguous)
