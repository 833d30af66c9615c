"""Acceptance of candidate draws: fixed threshold or empirical q-quantile.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 2.2 and Appendix A part C accept an assignment iff M <= a.  Section 2.2 also lets
the user give an acceptance probability q instead ("retaining the best 1%"), and its
planning example keeps exactly q*N of N draws (1e5 -> 1000, 2e5 -> 2000 at q = 0.01).
The reading implemented here:

* k = ceil(q * N * (1 - 1e-12)), clamped to [1, N]; the factor keeps a decimal q*N that
  is an integer (e.g. 0.01 * 2e5) from rounding up to the next count.
* Order draws by M.  Let t be the k-th smallest M, L = {M < t (1 - eps)} and
  E = {|M - t| <= eps * t} with eps = 1e-10.  Accept L and the k - |L| smallest keys of
  E.  Values within eps of each other (for example M(w) and M(1 - w) when n1 = n / 2,
  equal in exact arithmetic) are thus ordered by key, not by rounding noise.
"""

import math

import numpy as np

EPS_TIE = 1e-10
Q_FUZZ = 1e-12


def quantile_count(q, N):
    if not (0.0 < q <= 1.0) or N < 1:
        raise ValueError("q must be in (0, 1] and N >= 1")
    k = math.ceil(q * N * (1.0 - Q_FUZZ))
    return int(min(max(k, 1), N))


def accept_quantile(keys, M, k, eps=EPS_TIE):
    """Accepted keys (ascending) under the tie rule above."""
    keys = np.asarray(keys, dtype=np.uint64)
    M = np.asarray(M, dtype=np.float64)
    if not 1 <= k <= len(M):
        raise ValueError("k out of range")
    t = np.sort(M)[k - 1]
    low = M < t * (1.0 - eps)
    near = np.abs(M - t) <= eps * t
    need = k - int(low.sum())
    near_keys = np.sort(keys[near])
    chosen = np.concatenate([keys[low], near_keys[:need]])
    return np.sort(chosen)


def accept_threshold(keys, M, a):
    keys = np.asarray(keys, dtype=np.uint64)
    M = np.asarray(M, dtype=np.float64)
    return np.sort(keys[M <= a])
