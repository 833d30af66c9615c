"""The oracle's end-to-end calls, chained as the library chains them.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Pool generation (section 2.3, ``generate_randomizations``; section 2.1, "Batched
processing" and "Key-only storage"): draw candidate assignments in batches, compute M for
each, accept by threshold or by q-quantile, keep the keys of accepted draws.  Inference
(section 2.3, ``randomization_test``): regenerate accepted assignments from their keys and
run the conditional randomization test.  Batches of ``batch`` draws (the paper's snippet
uses batch_size = 1e4, Appendix B) bound memory; batching does not change any result.
"""

from math import comb

import numpy as np

from . import accept, assign, balance, frt, prep


def balance_of_keys(X, n1, ridge_rel, seed, keys, exact=False, batch=10000, metric="mahalanobis"):
    """M (FP64, textbook form) of the draws with the given keys."""
    P = prep.prepare(X, n1, ridge_rel, metric)
    n = P["n"]
    keys = np.asarray(keys, dtype=np.uint64)
    out = np.empty(len(keys), dtype=np.float64)
    for s in range(0, len(keys), batch):
        kb = keys[s:s + batch]
        if exact:
            W = np.stack([assign.exact_assignment(int(r), n, n1) for r in kb])
        else:
            W = assign.mc_assignments_batch(seed, kb, n, n1)
        if metric == "max_smd":
            out[s:s + batch] = balance.max_smd_batch(X, W, np.diag(P["S_lam"]))
        else:
            out[s:s + batch] = balance.mahalanobis_batch(X, W, P["S_lam"])
    return out


def draw_balance(X, n1, ridge_rel, seed, key_begin, num_draws, mode, q_or_a,
                 batch=10000, metric="mahalanobis"):
    """Monte Carlo pool: returns (accepted keys ascending, their M, M of every draw)."""
    keys = np.arange(key_begin, key_begin + num_draws, dtype=np.uint64)
    M = balance_of_keys(X, n1, ridge_rel, seed, keys, batch=batch, metric=metric)
    return _accept(keys, M, mode, q_or_a) + (M,)


def draw_exact(X, n1, ridge_rel, mode, q_or_a):
    """Exact enumeration over all C(n, n1) colex ranks."""
    n = np.asarray(X).shape[0]
    keys = np.arange(comb(n, n1), dtype=np.uint64)
    M = balance_of_keys(X, n1, ridge_rel, 0, keys, exact=True)
    return _accept(keys, M, mode, q_or_a) + (M,)


def _accept(keys, M, mode, q_or_a):
    if mode == "quantile":
        k = accept.quantile_count(q_or_a, len(keys))
        acc = accept.accept_quantile(keys, M, k)
    elif mode == "threshold":
        acc = accept.accept_threshold(keys, M, q_or_a)
    else:
        raise ValueError(mode)
    pos = np.searchsorted(keys, acc)
    return acc, M[pos]


def regenerate(seed, keys, n, n1, exact=False):
    keys = np.asarray(keys, dtype=np.uint64)
    if exact:
        return np.stack([assign.exact_assignment(int(r), n, n1) for r in keys])
    return assign.mc_assignments_batch(seed, keys, n, n1)


def rand_test_keys(seed, keys, n, n1, obs_index, Y, taus, exact=False):
    W = regenerate(seed, keys, n, n1, exact)
    return frt.rand_test(W, obs_index, Y, taus)
