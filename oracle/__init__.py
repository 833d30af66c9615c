"""CPU oracle for rerandomization with key-only storage (Goldstein, Jerzak, Kamat & Zhu,
"FastRerandomize: Fast Rerandomization Using Accelerated Computing").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package: only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

The oracle is a plain, slow, FP64 / exact-integer implementation of what the hot path
computes, written from the paper's definitions in the paper's order:

* ``philox``   -- the counter-based generator named for per-draw streams (published
                  definition, SC'11), in Python integers and a vectorised NumPy copy.
* ``assign``   -- draw key -> unit keys -> the n1 smallest -> treatment indicator;
                  colex unranking for exact enumeration; bitmask packing.
* ``prep``     -- sample covariance, ridge, Cholesky feasibility check (whitening,
                  section 2.2 and the Appendix A remark on general Sigma_X).
* ``balance``  -- the Mahalanobis statistic in its textbook form
                  M = (n1 n0 / n) (xbar_T - xbar_C)^T S^-1 (xbar_T - xbar_C).
* ``accept``   -- acceptance at a threshold a or at the empirical q-quantile of M.
* ``frt``      -- randomization test conditioned on acceptance, with exact rational
                  arithmetic, over a grid of sharp nulls tau0 (fiducial interval).
* ``diagnose`` -- closed forms of section 2.2 / Appendix A (chi-square truncation
                  factor v_a(d), RMSE, design-stage inversion for q).
* ``pipeline`` -- the above chained as the library calls chain them.

The oracle shares no code with the HIP library; the only module both sides use is the
seeded input generator ``paper_2501_07642_amd.inputs`` (no method arithmetic there).
"""

from . import philox, assign, prep, balance, accept, frt, diagnose, pipeline  # noqa: F401
