/*
 * rr.h -- C ABI of the MI355X (gfx950) rerandomization library, librr.so.
 *
 * The library implements the data-parallel hot path of rerandomization with key-only
 * storage as described in Goldstein, Jerzak, Kamat & Zhu, "FastRerandomize: Fast
 * Rerandomization Using Accelerated Computing":
 *   - whitening of the covariates (section 2.2; Appendix A remark on general Sigma_X),
 *   - batched candidate generation, balance evaluation and acceptance, keeping only the
 *     keys of accepted draws (section 2.1 "Batched processing", "Key-only storage";
 *     section 2.3 generate_randomizations),
 *   - the randomization test conditioned on acceptance over a grid of sharp nulls
 *     (section 2.3 randomization_test; section 4 "Design-based inference").
 *
 * Conventions shared by every call
 *   - Pointers named d_* are device pointers (HBM of the current HIP device); pointers
 *     named h_* are host pointers.  The caller owns all of them.
 *   - `stream` is a hipStream_t passed as void* (0 = the null stream).  Calls enqueue their
 *     kernels on it and return after the work has completed (they synchronise the stream
 *     when a data-dependent size must be known on the host), so outputs are ready on return;
 *     the exceptions, rr_draw_balance_async and rr_balance_keys_noalloc, only enqueue.
 *   - On any error nothing is written to the outputs, except RR_E_CAPACITY, which writes
 *     the required count to *h_count.  rr_last_error() returns a message for the last
 *     failing call of the calling thread.
 *   - A handle (rr_problem) owns its device workspace; it is not thread-safe: use one
 *     handle per host thread / stream.
 *
 * The balance statistic is reported on the chi^2_d scale,
 *     M(w) = (n1 n0 / n) (xbar_T - xbar_C)^T S_lam^-1 (xbar_T - xbar_C),
 * i.e. the paper's M = Delta^T Sigma_X^-1 Delta (section 2.2) divided by (1/n1 + 1/n0).
 */
#ifndef RR_H
#define RR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rr_problem rr_problem;

typedef enum {
    RR_OK = 0,
    RR_E_ARG = 1,        /* invalid argument (sizes, null pointers, q outside (0,1], ...) */
    RR_E_SINGULAR = 2,   /* covariance not positive definite after the ridge */
    RR_E_CAPACITY = 3,   /* output capacity too small; *h_count holds the required count */
    RR_E_RANGE = 4,      /* value outside the exactly representable range (see call) */
    RR_E_OBS = 5,        /* observed-assignment index not among the accepted keys */
    RR_E_DEVICE = 6,     /* HIP runtime error (message in rr_last_error) */
    RR_E_UNSUPPORTED = 7 /* shape beyond this build's limits (see call) */
} rr_status;

enum { RR_MODE_QUANTILE = 0, RR_MODE_THRESHOLD = 1, RR_MODE_CHI2_QUANTILE = 2 };
enum { RR_PREC_SPLIT_BF16 = 0, RR_PREC_FP32 = 1, RR_PREC_FIXED_I8 = 2, RR_PREC_GRAM_BF16 = 3 };
enum { RR_X_FP64 = 0, RR_X_FP32 = 1 };
enum { RR_METRIC_MAHALANOBIS = 0, RR_METRIC_DIAGONAL = 1, RR_METRIC_MAX_SMD = 2 };

/* Largest unit count of a Monte Carlo problem in this build. */
#define RR_MAX_N 4096
/* Largest unit count for exact enumeration (bitmask of one 64-bit word). */
#define RR_MAX_N_EXACT 64
/* Largest covariate count: one LDS stage of the contraction's operand records stays within
 * a 2^31-byte buffer range. */
#define RR_MAX_D (1 << 22)

/*
 * rr_prepare -- whitening and workspace set-up (section 2.2: covariates whitened so that
 * Sigma_X = I; Appendix A remark: X~ = X Sigma^-1/2 gives M = ||Delta~||^2).
 *
 *   d_X      device, n rows x d columns, row-major with leading dimension ldx >= d,
 *            FP64 (x_dtype = RR_X_FP64) or FP32 (RR_X_FP32, promoted to FP64).
 *   n1       treated-group size, 1 <= n1 <= n-1.  n <= RR_MAX_N, 1 <= d <= RR_MAX_D.
 *   ridge_rel  lambda = ridge_rel * tr(S) / d is added to the diagonal of the sample
 *            covariance S (denominator n - 1) before the Cholesky factorisation; >= 0.
 *            With d >= n - 1, S is singular and ridge_rel > 0 is required.
 *   out      receives the handle.
 * Computes on the device, in FP64: column means mu, S, S_lam = S + lambda I, its
 * Cholesky factor L, the whitened centred covariates X~ = (X - 1 mu^T) L^-T, and from X~
 * the BF16 hi/lo and FP32 operand copies used by rr_draw_*.
 * Errors: RR_E_ARG, RR_E_SINGULAR (a pivot <= 0, or min L_jj^2 < 1e-10 max S_jj),
 * RR_E_UNSUPPORTED (n > RR_MAX_N or d > RR_MAX_D), RR_E_DEVICE.
 */
rr_status rr_prepare(const void* d_X, int x_dtype, int64_t n, int64_t d, int64_t ldx,
                     int64_t n1, double ridge_rel, void* stream, rr_problem** out);

/*
 * rr_prepare_metric -- rr_prepare with a choice of balance metric.
 *   metric = RR_METRIC_MAHALANOBIS: as rr_prepare (whitening by the Cholesky factor).
 *   metric = RR_METRIC_DIAGONAL: the covariates are standardised but not decorrelated:
 *            S_lam is replaced by its diagonal, so M = (n1 n0 / n) sum_j Delta_j^2 /
 *            (S_jj + lambda), the sum of squared standardised mean differences (section 2.2
 *            states M for standardised covariates).  Every later call is unchanged.
 *   metric = RR_METRIC_MAX_SMD: the per-column criterion: the same standardisation, and the
 *            balance value of a draw is the largest squared standardised mean difference,
 *            M = (n1 n0 / n) max_j Delta_j^2 / (S_jj + lambda) (section 2.2 writes M as the sum
 *            of the squared SMD_j; this scores the worst covariate instead, on the chi^2_1 scale
 *            of each term).  Acceptance, outputs and the guard band work on this value; the
 *            Gram form has no per-column sums and is rejected with it (RR_E_ARG).
 * Errors as rr_prepare (RR_E_SINGULAR: some S_jj + lambda <= 1e-10 max S_jj); RR_E_ARG for an
 * unknown metric.
 */
rr_status rr_prepare_metric(const void* d_X, int x_dtype, int64_t n, int64_t d, int64_t ldx,
                            int64_t n1, double ridge_rel, int metric, void* stream,
                            rr_problem** out);

/* Releases a handle and its device memory.  Null is ignored. */
void rr_free(rr_problem* p);

/* Message of the last error of the calling thread ("" if none). */
const char* rr_last_error(void);

/* Read-only views of a prepared problem (host values). */
int64_t rr_problem_n(const rr_problem* p);
int64_t rr_problem_d(const rr_problem* p);
int64_t rr_problem_n1(const rr_problem* p);
double rr_problem_lambda(const rr_problem* p);

/*
 * rr_draw_balance -- Monte Carlo pool generation with key-only storage (section 2.3
 * generate_randomizations with randomization_type = "monte_carlo"; section 2.1).
 *
 * Draw keys are the integers b in [key_begin, key_begin + num_draws).  Draw b treats the
 * n1 units with the smallest (u_i, i), where u_i is word (i/64) mod 4 of Philox-4x32-10
 * block 64*(i/256) + i%64 under counter (block, 0, lo32(b), hi32(b)) and key
 * (lo32(seed), hi32(seed)).  M is computed for every draw; the accepted draws are
 *   mode = RR_MODE_THRESHOLD: those with M <= q_or_a (section 2.2, Appendix A part C);
 *   mode = RR_MODE_CHI2_QUANTILE: those with M <= c_q, the q-quantile of chi^2_d for
 *     q = q_or_a in (0, 1] (section 2.2: the threshold a_q taken from the chi-square
 *     approximation of M; rr_diagnose reports the same c_q);
 *   mode = RR_MODE_QUANTILE:  k = ceil(q N (1 - 1e-12)) draws with the smallest M
 *     (section 2.2, acceptance probability q), q = q_or_a in (0, 1]; values within a
 *     relative 1e-10 of the k-th smallest are ordered by key.
 * precision selects the operand format of the W X~ contraction: RR_PREC_SPLIT_BF16
 * (X~ = hi + lo in BF16, FP32 accumulation), RR_PREC_FP32, or RR_PREC_FIXED_I8 (X~ in
 * 15-bit fixed point per block of 32 covariates, x = s (128 hi + lo) with int8 digits,
 * summed exactly in int32 on the int8 matrix cores), or RR_PREC_GRAM_BF16 (the Gram form
 * M = n/(n1 n0) w^T (X~ X~^T) w: the n x n Gram matrix split into BF16 hi + lo, n^2 instead
 * of n d work per draw, for d > n; the Gram operands are built on the first call that asks
 * for them).  Every draw whose FP32 value is not provably on one side of the acceptance
 * boundary is recomputed in FP64, so the accepted set does not depend on the precision.
 *
 * Outputs (device, caller-allocated, `capacity` entries):
 *   d_keys   accepted keys, ascending;
 *   d_M      their M: the FP64 recomputation for draws of the guard band and, when d <= 64
 *            or precision = RR_PREC_FIXED_I8 or RR_PREC_GRAM_BF16, for every accepted draw (the BF16 hi + lo
 *            representation of X~ limits the FP32 value's relative accuracy to about
 *            2^-17 sqrt(d / M), the fixed-point one to about 2^-13 sqrt(d / M)); else the
 *            FP32 value, within 1e-4 relative;
 *   d_flags  optional (may be null): 1 where d_M holds the FP64 recomputation.
 *   h_count  host: number of accepted draws.
 * Errors: RR_E_ARG, RR_E_CAPACITY, RR_E_DEVICE.
 */
rr_status rr_draw_balance(rr_problem* p, uint64_t seed, uint64_t key_begin,
                          uint64_t num_draws, int mode, double q_or_a, int precision,
                          uint64_t* d_keys, double* d_M, uint8_t* d_flags,
                          uint64_t capacity, uint64_t* h_count, void* stream);

/*
 * rr_draw_balance_async -- rr_draw_balance, stream-ordered: the call enqueues all its work on
 * `stream` (and on the handle's internal generation stream, joined to it by events) and
 * returns without waiting.  The accepted count and the status are written on the device:
 *   d_count   device, 1 uint64: the accepted count K (on RR_E_CAPACITY, the required count);
 *   d_status  device, 1 int32: RR_OK, or the rr_status the synchronous call would have
 *             returned for a condition detected on the device (RR_E_CAPACITY,
 *             RR_E_UNSUPPORTED for a candidate or guard-band list beyond its capacity,
 *             RR_E_DEVICE for an inconsistent selection).
 * Results are identical to rr_draw_balance; on a device-detected error nothing is written to
 * d_keys / d_M / d_flags.  Arguments checked on the host are returned as usual (with
 * RR_E_CAPACITY for q N above the capacity, the count is also written to d_count).  The
 * caller synchronises `stream` before reading any output.  Differences: the autotuner is not
 * run (its cached choice or the default tile is used), rr_last_timing is not updated, and a
 * call that must grow the handle's workspace, or build the Gram operands, waits for the work
 * in flight first.  Successive calls on one handle and stream are ordered by the stream.
 */
rr_status rr_draw_balance_async(rr_problem* p, uint64_t seed, uint64_t key_begin,
                                uint64_t num_draws, int mode, double q_or_a, int precision,
                                uint64_t* d_keys, double* d_M, uint8_t* d_flags,
                                uint64_t capacity, uint64_t* d_count, int32_t* d_status,
                                void* stream);

/*
 * rr_draw_exact -- exact enumeration (section 2.3, randomization_type = "exact"): every
 * assignment is drawn once; its key is its colex rank r = sum_t C(i_t, t) over the treated
 * indices i_1 < ... < i_n1, r in [0, C(n, n1)).  Acceptance and outputs as in
 * rr_draw_balance.  Requires n <= RR_MAX_N_EXACT and C(n, n1) < 2^40 (RR_E_RANGE).
 */
rr_status rr_draw_exact(rr_problem* p, int mode, double q_or_a, int precision,
                        uint64_t* d_keys, double* d_M, uint8_t* d_flags,
                        uint64_t capacity, uint64_t* h_count, void* stream);

/*
 * rr_regenerate -- assignments from keys (section 2.1 "Key-only storage": the PRNG
 * regenerates an accepted assignment from its key on demand).
 *   d_keys     device, K keys (draw indices, or colex ranks when exact != 0);
 *   d_bits     device, K x ceil(n/32) uint32: bit (i % 32) of word i/32 of row k is 1 iff
 *              unit i is treated in draw k.
 */
rr_status rr_regenerate(rr_problem* p, uint64_t seed, int exact, const uint64_t* d_keys,
                        uint64_t K, uint32_t* d_bits, void* stream);

/*
 * rr_balance_keys -- M of given draws by both device paths, for verification.
 *   d_M32, d_err  device, K floats each (may be null): the FP32 value of the contraction
 *                 in the given precision (any RR_PREC_*, as for rr_draw_balance) and its
 *                 rigorous error bound, so |M32 - M| <= err;
 *   d_M64         device, K doubles (may be null): the FP64 recomputation.
 */
rr_status rr_balance_keys(rr_problem* p, uint64_t seed, int exact, const uint64_t* d_keys,
                          uint64_t K, int precision, float* d_M32, float* d_err,
                          double* d_M64, void* stream);

/*
 * rr_balance_keys_noalloc -- rr_balance_keys for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, outputs and results as rr_balance_keys, but:
 *   - its scratch is a fixed 64 MiB array in the library's device memory (one per GPU, held
 *     until the process ends) instead of the handle's workspace, so it calls no hipMalloc /
 *     hipFree / allocating routine; K is limited to (2^26 - 256) / (32 S) keys when d_M32 is
 *     set (S = ceil(n/256) rounded up to a power of two: 524286 keys at n <= 1024), else
 *     RR_E_UNSUPPORTED with the limit in rr_last_error();
 *   - it only enqueues kernels on `stream` and returns without synchronising: outputs are
 *     ready once the stream has reached that point;
 *   - every call on a GPU shares that GPU's scratch array: calls that overlap on one GPU (on
 *     different streams or threads) race and must be ordered by the caller;
 *   - the current device must be the handle's (RR_E_ARG otherwise), and RR_PREC_GRAM_BF16
 *     needs the handle's Gram operands built by an earlier allocating call (RR_E_ARG).
 */
rr_status rr_balance_keys_noalloc(rr_problem* p, uint64_t seed, int exact, const uint64_t* d_keys,
                                  uint64_t K, int precision, float* d_M32, float* d_err,
                                  double* d_M64, void* stream);

/*
 * rr_rand_test -- randomization test conditioned on acceptance (section 2.3
 * randomization_test; section 4 "Design-based inference").
 *
 *   d_keys, K    the accepted keys (device); the observed assignment is key d_keys[obs_index].
 *   d_Y          device, n observed outcomes (FP64).
 *   h_tau0, G    host, G sharp-null effects tau0 (H0: Y_i(1) - Y_i(0) = tau0 for all i).
 *   d_counts     device, G uint64: c_g = #{k : |T_k(tau0_g)| >= |T_obs(tau0_g)|}, where
 *                T_k(tau0) is the difference in means of Y - tau0 * w_obs under draw k;
 *                the p-value is c_g / K (>= 1/K since w_obs is among the draws).
 *   h_tau_hat    host (may be null): observed difference in means.
 * The statistic is evaluated exactly on Y rounded to the grid 2^-s, s = 61 - t - e with
 * n^2 <= 2^t and max|Y| = f 2^e, f in [0.5, 1).  RR_E_RANGE if a tau0 is too large or too
 * finely resolved for the 128-bit comparison (|tau0| >= 2^-8 and |tau0| < 2^20 are
 * always accepted, as is tau0 = 0); RR_E_OBS if obs_index >= K.
 */
rr_status rr_rand_test(rr_problem* p, uint64_t seed, int exact, const uint64_t* d_keys,
                       uint64_t K, uint64_t obs_index, const double* d_Y,
                       const double* h_tau0, int64_t G, uint64_t* d_counts,
                       double* h_tau_hat, void* stream);

/*
 * rr_rand_test_interval -- rr_rand_test plus the fiducial interval obtained by inverting the
 * test over the null grid (section 2.3: randomization_test's optional inversion returns a
 * fiducial interval; section 4).  The paper fixes neither the level nor the shape; here the
 * interval is the set of grid values tau0_g whose p-value c_g / K exceeds alpha:
 *   h_interval   host, 2 doubles: [min, max] of those tau0_g (both NaN when none is kept);
 *   h_contiguous host: 1 when the kept grid points are contiguous in the caller's grid order
 *                (or none is kept), 0 when the kept set has gaps (a non-convex region).
 * Other arguments and outputs as rr_rand_test; G >= 1 and 0 < alpha < 1 (RR_E_ARG otherwise).
 */
rr_status rr_rand_test_interval(rr_problem* p, uint64_t seed, int exact, const uint64_t* d_keys,
                                uint64_t K, uint64_t obs_index, const double* d_Y,
                                const double* h_tau0, int64_t G, double alpha,
                                uint64_t* d_counts, double* h_tau_hat, double* h_interval,
                                int* h_contiguous, void* stream);

/*
 * rr_draw_balance_batched -- many independent Monte Carlo pools in one persistent launch
 * (section 2.1 "Batched processing").  Problem i uses handle P[i], seed seeds[i], draws
 * [key_begin, key_begin + num_draws) and the same mode / q_or_a / precision for all.
 * Outputs: d_keys[i], d_M[i] (device pointers, capacity entries each) and h_counts[i].
 * Results are identical to nprob calls of rr_draw_balance.
 */
rr_status rr_draw_balance_batched(rr_problem* const* P, int64_t nprob, const uint64_t* seeds,
                                  uint64_t key_begin, uint64_t num_draws, int mode,
                                  double q_or_a, int precision, uint64_t* const* d_keys,
                                  double* const* d_M, uint64_t capacity, uint64_t* h_counts,
                                  void* stream);

/*
 * Design diagnostics (host computation, no device work): closed forms for choosing the
 * acceptance probability q (section 2.2; Appendix A parts A-D), for n1 treated and n0
 * control units, d whitened covariates, outcome noise sd sigma and R^2 of the outcome on
 * the covariates (0 <= r2 < 1).  M is taken as chi^2_d under complete randomization.
 */
typedef struct {
    double c_q;            /* q-quantile of chi^2_d: acceptance threshold on the scale of M */
    double a_q;            /* the same threshold on the paper's scale, (1/n1 + 1/n0) c_q */
    double v_a;            /* Pr(chi^2_{d+2} <= c_q) / Pr(chi^2_d <= c_q): variance shrinkage of
                              each whitened covariate mean difference (Appendix A part C) */
    double expected_M;     /* E[M | accepted] = d v_a */
    double rmse_reduction; /* 1 - sqrt((1 + v_a s) / (1 + s)), s = r2 / (1 - r2) */
    double mse_complete;   /* (1/n1 + 1/n0)(sigma^2 + s sigma^2): complete randomization */
    double mse_accept;     /* (1/n1 + 1/n0)(sigma^2 + v_a s sigma^2): conditional on acceptance */
} rr_design;

/* Closed forms at acceptance probability q in (0, 1] (q = 1: c_q = inf, v_a = 1).
 * Errors: RR_E_ARG (n1, n0, d < 1, sigma <= 0, r2 outside [0, 1), q outside (0, 1]). */
rr_status rr_diagnose(int64_t n1, int64_t n0, int64_t d, double q, double sigma, double r2,
                      rr_design* out);

/* q* (Appendix A part D): the largest q with mse_accept(q) <= tau^2 / (z_{1-alpha/2} +
 * z_power)^2, searched over [q_lo, 1] (mse_accept increases with q).  *q_star = 1 when q = 1
 * already meets the target.  Errors: RR_E_ARG; RR_E_RANGE when no q >= q_lo meets it. */
rr_status rr_q_star(int64_t n1, int64_t n0, int64_t d, double sigma, double r2, double tau,
                    double alpha, double power, double q_lo, double* q_star);

/* Realised RMSE of the difference in means for an accepted assignment with balance statistic M
 * (chi^2_d scale, as reported by rr_draw_balance), under the linear outcome model of section 2.2
 * with noise sd sigma and R^2 = r2, sigma_prog^2 = r2 / (1 - r2) sigma^2 and the paper's
 * imbalance ||Delta||^2 = (1/n1 + 1/n0) M (Appendix A part A):
 *   rmse_typical = sqrt(sigma^2 (1/n1 + 1/n0) + sigma_prog^2 ||Delta||^2 / d), the expected squared
 *                  bias over prognostic directions uniform on the sphere (typical orientation);
 *   rmse_bound   = sqrt(sigma^2 (1/n1 + 1/n0) + sigma_prog^2 ||Delta||^2), the Cauchy-Schwarz bound
 *                  (the prognostic direction aligned with the imbalance).
 * Errors: RR_E_ARG (as rr_diagnose; M negative or not finite). */
rr_status rr_realized_rmse(int64_t n1, int64_t n0, int64_t d, double M, double sigma, double r2,
                           double* rmse_typical, double* rmse_bound);

/* The autotuner's choices of this process (and of RR_TUNE_FILE, when set) as a JSON document:
 * {"rr_tune": [{"batched": B, "prec": P, "S": S, "cost_log2": C, "db": D, "gen_wg": G,
 * "chunk_log2": L, "ms": T}, ...]}, one entry per single-pool bucket (batched = 0: precision,
 * 256-unit chunks per draw S, floor(log2(K steps x covariate blocks))) or batched class
 * (batched = 1, cost_log2 = -1; read from RR_TUNE_FILE only, batched calls do not probe):
 * contraction tile db (32-draw blocks per wave), generation workgroups per CU, draws per
 * pipeline chunk 2^L, and the probe's time.  Writes at most len
 * bytes (NUL-terminated) to the host buffer buf; *needed (may be null) receives the size
 * required.  RR_E_CAPACITY when len is too small, RR_E_ARG for a null buffer. */
rr_status rr_tune_report(char* buf, uint64_t len, uint64_t* needed);

/* Timing of the last rr_draw_balance / rr_draw_exact / rr_draw_balance_batched call on
 * this thread: host wall milliseconds of the call, and HIP-event milliseconds summed over the
 * launches of the contraction kernel (on the caller's stream) and of the generation kernel
 * (on the handle's internal stream, overlapping the contraction); number of chunks (launches
 * of each kernel); size of the FP64-rechecked guard band.  All pointers may be null. */
rr_status rr_last_timing(double* total_ms, double* contract_ms, double* gen_ms,
                         int64_t* draw_launches, uint64_t* band_size);

#ifdef __cplusplus
}
#endif

#endif /* RR_H */
