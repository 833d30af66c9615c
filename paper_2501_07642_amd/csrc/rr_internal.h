// Internal declarations of librr: problem handle, device helpers shared by the kernels.
//
// Target: gfx950 (CDNA4), wave64.  Every kernel is written for 64-lane wavefronts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rr.h"

namespace rr {

// ---------------------------------------------------------------------------------------
// Error plumbing (host).
void set_error(const std::string& msg);
#define RR_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ::rr::set_error(std::string(#call) + ": " + hipGetErrorString(e_));        \
            return RR_E_DEVICE;                                                        \
        }                                                                              \
    } while (0)

// ---------------------------------------------------------------------------------------
// Layout constants.
constexpr int kWave = 64;
constexpr int kUnitsPerChunk = 256;   // one Philox block per lane yields 4 x 64 units
constexpr int kKStep = 16;            // units per MFMA K step (32x32x16 BF16)
constexpr int kKStepsPerStage = 8;    // K steps per LDS stage of the contraction
constexpr int kColBlock = 32;         // covariates per MFMA row block
constexpr int kRecordU4 = 128;        // uint4 per operand record: 2 planes x 64 lanes x 16 B
constexpr int kRecordU4I8 = 64;       // fixed-point int8 records: 1 plane x 64 lanes x 16 B
// Fixed-point digits: x = s (128 hi + lo), hi in [-127, 127], lo in [-64, 63], so the
// quantised value q = 128 hi + lo spans [-16320, 16319] and s = max|x| / kQMax per block.
constexpr int kQMax = 16319;
constexpr int kQMin = -16320;
constexpr int kMaxS = RR_MAX_N / kUnitsPerChunk;   // 16
// Zeroed doubles after X~ (n x d, row-major): the FP64 recheck's lanes for columns past d
// read up to 15 values beyond the end of their row, which for the last row lands here.
constexpr int64_t kX64Pad = 16;
constexpr uint32_t kXcds = 8;          // accelerator dies; workgroups are dealt to them round robin

// Position of workgroup b inside each grid-stride window of g items, such that the g / 8
// workgroups on one XCD (b mod 8) take neighbouring items: a permutation of [0, g) when g is a
// multiple of 8, else the identity.
__host__ __device__ inline uint32_t xcd_slot(uint32_t b, uint32_t g) {
    return g % kXcds == 0 ? (b % kXcds) * (g / kXcds) + b / kXcds : b;
}

// Host-side description of a prepared problem.
struct Problem {
    int device = 0;
    uint64_t uid = 0;      // unique per prepared problem in this process (never reused)
    int64_t n = 0, d = 0, n1 = 0, n0 = 0;
    double ridge_rel = 0, lambda = 0;
    int metric = RR_METRIC_MAHALANOBIS;
    int S = 0;             // 256-unit chunks per draw: ceil(n / 256)
    int wstride = 0;       // uint32 words per draw bitmask in the internal layout: 8 * S
    int64_t ks = 0;        // K steps of 16 units, a multiple of kKStepsPerStage (units >= n are zero)
    int64_t ncb = 0;       // covariate blocks of 32 (padded)
    double scale = 0;      // n / (n1 n0)
    // device buffers (X64 .. bscale and cabs are carved from one allocation, mem)
    void* mem = nullptr;
    double* X64 = nullptr;     // n x d whitened, centred covariates X~ (FP64, row-major)
    double* L = nullptr;       // d x d Cholesky factor of S_lam (lower)
    double* mu = nullptr;      // d column means
    uint4* op_split = nullptr; // ks * ncb records: BF16 hi / lo planes
    uint4* op_f32 = nullptr;   // ks * ncb records: FP32 planes
    uint4* op_i8 = nullptr;    // ks * ncb records: fixed-point int8 digits (one plane)
    float* bscale = nullptr;   // ncb fixed-point scales s, one per block of 32 covariates
    double qerr_c2 = 0;        // sum_j e_j^2, e_j bounding the fixed-point error of G_j (host)
    // Gram form (built on first use): records of K = X~ X~^T in the split layout, its units
    // taking the place of the covariates
    uint4* op_gram = nullptr;  // ks * ncb_gram records: BF16 hi / lo planes of K
    int64_t ncb_gram = 0;      // blocks of 32 units (padded to whole chunks)
    double gram_ctop = 0;      // sum of the n1 largest column sums of |K| (host, error bound)
    float* cabs = nullptr;     // 32 * ncb column sums of |X~| (rounded up; 0 for pads)
    double cabs_c2 = 0;        // sum of cabs^2 (host copy, for the error bound)
    double cabs_max = 0;       // max of cabs (host copy, bound of the per-column criterion)
    // bounds e_j of |G32_j - G_j| over the covariates (host): sum of squares and largest, for
    // the split BF16 and FP32 contractions
    double esplit_n2 = 0, esplit_max = 0, ef32_n2 = 0, ef32_max = 0;
    double qerr_max = 0;       // max_j e_j of the fixed-point form (host)
    // workspace for the draw pipeline (grown on demand)
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // workspace of rr_balance_keys and rr_rand_test (grown on demand, kept with the handle)
    void* aux = nullptr;
    size_t aux_bytes = 0;
    hipStream_t gen_stream = nullptr;     // internal stream of the generation kernels
    std::vector<hipEvent_t> events;       // chunk ordering and timing
    hipStream_t events_stream = nullptr;  // the caller's stream the events were last recorded on
    struct BatchState* batch = nullptr;   // batched-call resources when this handle leads a batch
};
void free_batch_state(Problem& P);
// Grows the handle's auxiliary workspace to at least `bytes` (device memory kept until rr_free).
rr_status ensure_aux(Problem& P, size_t bytes);


// ---------------------------------------------------------------------------------------
// Kernel argument blocks (shared by the kernels and the pipeline).
struct GenArgs {
    uint64_t seed, key_begin, num;
    const uint64_t* keylist;  // non-null: keys of the draws; else key_begin + index
    const uint64_t* binom;    // exact mode: C(i, t), i <= 64, t <= 32
    int n, n1;
    uint32_t* out;            // 8 S words per draw
};

struct ContractArgs {
    const uint32_t* bits;     // 8 S words per draw (from the generation kernel)
    uint64_t num;             // draws in this launch
    uint64_t key_begin;       // key of draw i is key_begin + i, or keylist[i]
    const uint64_t* keylist;
    const uint4* op;          // operand records, ks * ncb records of kRecordU4 uint4
    const float* cabs;        // 32 * ncb
    const float* bscale;      // fixed-point form: scale of each block of 32 covariates
    int n, ks, ncb;
    float scale;              // n / (n1 n0)
    float two_kappa;          // 2 * kappa: |G32_j - G_j| <= kappa * cabs_j
    float csq;                // kappa^2 * sum_j cabs_j^2
    float cnorm;              // ||cabs||_2, rounded up
    float gamma_ss;           // relative bound of the FP32 sum of squares and the scaling
    float safety;             // multiplies the assembled bound
    int maxmode;              // 1: M = scale max_j G_j^2 (per-column criterion), else scale sum_j G_j^2
    const float* U;           // append iff lo <= *U; null appends every draw
    uint64_t* cand_key;
    float* cand_hi;
    float* cand_lo;
    float* cand_m;
    uint32_t* cand_count;
    uint32_t cand_cap;
    float* out_m32;           // evaluation mode (with out_err) or dense mode (with out_hi / out_lo)
    float* out_err;           // evaluation mode: per-draw m32 and error bound, no prefilter
    float* out_hi;            // dense mode: per-draw upper / lower bounds and m32 at index i
    float* out_lo;
    // batched launches: tile t covers draws of problem tab[t / tpp], tile t % tpp
    const ContractArgs* tab;
    uint32_t tpp, nprob;
};

struct RecheckArgs {
    const double* X64;        // n x d, row-major
    const uint64_t* keys;     // keys of the draws
    const uint32_t* count;    // number of entries (device)
    uint32_t cap;             // entries past cap are ignored (the lists hold cap entries)
    uint64_t seed;
    const uint64_t* binom;
    int n, n1, d;
    double scale;
    double* out;              // M64 per entry
    int maxmode;              // 1: M = scale max_j G_j^2, else scale sum_j G_j^2
};

// Up to this many covariates every accepted draw is reported with its FP64 M: the BF16
// hi + lo representation error of X~ (2^-18 relative per entry) makes the FP32 value's
// relative error about 2^-17 sqrt(d / M), which can pass 1e-4 only at small d and tiny M.
constexpr int kRefineMaxD = 64;

inline bool valid_prec(int prec) {
    return prec == RR_PREC_SPLIT_BF16 || prec == RR_PREC_FP32 || prec == RR_PREC_FIXED_I8 ||
           prec == RR_PREC_GRAM_BF16;
}
// Accepted draws reported with their FP64 M: small d (see above), the fixed-point form, whose
// 15-bit representation of X~ leaves the FP32 value about 2^-13 sqrt(d / M) relative, and the
// Gram form, whose sum w^T K w can cancel (its FP32 value has no relative bound).
inline bool refine_accepted(const Problem& P, int prec) {
    return P.d <= kRefineMaxD || prec == RR_PREC_FIXED_I8 || prec == RR_PREC_GRAM_BF16;
}
// Builds the Gram-form operands of a prepared problem if they are missing (stream-ordered,
// synchronises the stream once).
rr_status ensure_gram(Problem& P, hipStream_t st);

// Launch configuration of the draw pipeline, chosen by the autotuner per problem bucket:
// draws per wave block of the contraction tile (db, 1 or 2) and generation workgroups per CU.
struct Tune {
    int db;                // 32-draw blocks per contraction wave
    int gen_wg;            // generation workgroups per CU
    int chunk_log2 = 20;   // draws per pipeline chunk (single-pool calls): 2^chunk_log2
};
// Generation workgroups per CU by default: three 4-wave workgroups (<= 64 VGPRs per wave up to
// 1024 units) fit beside one 8-wave contraction workgroup (<= 168 VGPRs per wave, up to ~131 KB
// LDS) on every CU.
constexpr int kGenWgPerCu = 3;

// Rigorous error-bound constants of the FP32 contraction of a problem (see rr_select.hip).
struct Bound {
    float two_kappa, csq, cnorm, gamma_ss, safety;
};

// Acceptance bookkeeping of one pool (device).
struct AcceptState {
    uint32_t k;               // quantile mode: accepted count
    uint32_t nL;              // accepted outright (FP32 bounds below the boundary)
    uint32_t band_count;      // guard-band entries
    uint32_t acc_count;       // accepted entries written
    uint32_t guard_fail;      // band selection inconsistent
    uint32_t overflow;        // a list exceeded its capacity
    uint32_t done;            // batched pools: sorted outputs written on the device
};

}  // namespace rr

struct rr_problem {
    rr::Problem P;
};

namespace rr {
// Host functions shared by the translation units.
hipError_t launch_gen(int S, bool exact, const GenArgs& g, int grid, hipStream_t st);
hipError_t launch_gen_batch(int S, const GenArgs* tab, uint64_t nprob, uint64_t per, int grid, hipStream_t st);
hipError_t launch_contract(int S, int prec, int db, bool batch, const ContractArgs& a, int grid, hipStream_t st);
int contract_tile(int prec, int S, int db);
bool contract_db_ok(int prec, int S, int db);
int contract_db_default(int prec, int S);
int contract_kernel_vgprs(int prec, int S, int db, bool batch);
int contract_waves(int prec, int S);
int gen_kernel_vgprs(int S, bool batch);
int gen_wg_fit(int prec, int S, int db, bool batch);
int draw_cb(int prec, int S);
hipError_t launch_recheck(int S, bool exact, const RecheckArgs& a, int grid, hipStream_t st);
hipError_t launch_recheck_batch(int S, const RecheckArgs* tab, int nprob, uint32_t* offs, int grid, hipStream_t st);
int pow2_chunks(int n);
int device_cus(int dev);
const uint64_t* binom_table(int dev);
const uint64_t* binom_table_ready(int dev);
// M32 / error bound / M64 of given draws, enqueued on `st` with caller-provided scratch: `cnt`
// (one uint32) and `bits` (8 S words per draw when d_M32 is set).
rr_status balance_keys_enqueue(Problem& P, uint64_t seed, bool exact, const uint64_t* binom,
                               const uint64_t* d_keys, uint64_t K, int precision, float* d_M32,
                               float* d_err, double* d_M64, uint32_t* cnt, uint32_t* bits,
                               hipStream_t st);
Bound bound_constants(const Problem& P, int prec);
// Bounds of |G32_j - G_j| for column j from the per-column sums of the preparation: the
// step-weighted sum of |X~|, the sum of the per-half maxima and the representation residual
// (split), and sum |X~|, the step-weighted sum and the residual (FP32).
double split_column_bound(const Problem& P, double wsum_j, double halfmax_j, double resid_j);
double fp32_column_bound(const Problem& P, double cabs_j, double wsum_j, double resid_j);
ContractArgs make_contract_args(const Problem& P, int prec, const Bound& b);
Tune tune_default(int prec, int S, bool batch);
// probe = false: the cached choice or the default, never a timed probe (asynchronous calls).
Tune tune_for(Problem& P, int prec, bool exact, uint64_t work_draws, hipStream_t st, bool probe = true);
// Batched launches: the cached per-class choice (precision, S) measured inside the graph, if any;
// and recording one.
bool batch_tune_lookup(int prec, int S, Tune* out);
rr_status draw_pipeline(Problem& P, bool exact, uint64_t seed, uint64_t key_begin, uint64_t N, int mode,
                        double q_or_a, int prec, uint64_t* d_keys, double* d_M, uint8_t* d_flags,
                        uint64_t capacity, uint64_t* h_count, hipStream_t st, const Tune* tune,
                        uint64_t* d_count = nullptr, int32_t* d_status = nullptr);
hipError_t sort_accepted(const uint64_t* acc_key, const double* acc_m, const uint8_t* acc_flag, uint32_t n,
                         uint64_t* const sk[2], uint32_t* const si[2], uint64_t* out_key, double* out_m,
                         uint8_t* out_flag, hipStream_t st, const uint32_t* n_dev = nullptr,
                         const int32_t* status = nullptr);
double chi2_quantile_of(double q, double d);   // q-quantile of chi^2_d (inf for q = 1)
void set_timing(double total_ms, double contract_ms, double gen_ms, int64_t launches, uint64_t band);
}  // namespace rr

namespace rr {

// ---------------------------------------------------------------------------------------
// Philox-4x32-10 (Salmon et al., SC'11): counter (c0..c3), key (k0, k1); per round the
// products M0*c0 and M1*c2 give (hi1^c1^k0, lo1, hi0^c3^k1, lo0); the key advances by the
// Weyl constants between rounds.
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// 32 x 32 -> 64-bit product in one v_mad_u64_u32 (left to itself the compiler splits some
// products into separate quarter-rate v_mul_lo_u32 / v_mul_hi_u32 instructions).
__device__ __forceinline__ uint64_t mul_wide(uint32_t a, uint32_t b) {
    uint64_t r, carry;
    asm("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(r), "=s"(carry) : "v"(a), "s"(b));
    (void)carry;
    return r;
}

__device__ __forceinline__ void philox_round(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                             uint32_t k0, uint32_t k1) {
    const uint64_t p0 = mul_wide(c0, kPhiloxM0);
    const uint64_t p1 = mul_wide(c2, kPhiloxM1);
    // three-input XOR in one gfx950 v_bitop3_b32 (truth table 0x96 = a ^ b ^ c)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
}

__device__ __forceinline__ void philox_block(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                             uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        philox_round(c0, c1, c2, c3, k0, k1);
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
}

// ---------------------------------------------------------------------------------------
// Wave helpers.
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// inclusive prefix sum across the wave
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (l >= o) v += t;
    }
    return v;
}

// Inclusive prefix sum across the wave without LDS traffic: shifted adds inside each 16-lane
// row through DPP (row_shr 1, 2, 4, 8; lanes shifted in from outside the row read 0), then
// the totals of the lower rows, read from lanes 15, 31 and 47 into scalar registers.
__device__ __forceinline__ uint32_t wave_incl_scan_rows(uint32_t v) {
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);
    const int t0 = __builtin_amdgcn_readlane(x, 15), t1 = __builtin_amdgcn_readlane(x, 31),
              t2 = __builtin_amdgcn_readlane(x, 47);
    const int lane = lane_id();
    x += (lane >= 16 ? t0 : 0) + (lane >= 32 ? t1 : 0) + (lane >= 48 ? t2 : 0);
    return (uint32_t)x;
}

// ---------------------------------------------------------------------------------------
// Monte Carlo draw: the n1 units with the smallest (u_i, i) become treated.  Unit
// i = 256 s + 64 r + lane reads word r of Philox block 64 s + lane under counter
// (block, 0, lo32(key), hi32(key)) and the pool seed as Philox key.
//
// Selection (exact): the n1-th smallest value u* is bracketed by [lo, hi] with
// #{u < lo} < n1 <= #{u <= hi}; counts come from wave ballots.  For n <= 2048 the first
// bracket is one top-byte bin of a 256-bin LDS histogram of the keys.  Pivots interpolate inside
// the bracket for the first steps (unit keys are uniform, so two or three steps leave a few
// values), then bisect, so the loop ends after at most 4 + 33 steps for any input.  The
// <= 64 values left in the bracket are ranked in LDS; values equal to u* are taken in unit
// order.  Output: bitmask words (bit i%32 of word i/32), written by lane 0 to `out` (8 S
// words).  `list` is a wave-private 128-entry LDS array (64 slots for the bracket values,
// 64 spare slots that take the non-members' stores).
//
// C > 0 fixes the number of 256-unit chunks (ceil(n / 256)) at compile time: the per-chunk
// validity tests fold away and only the last chunk keeps a runtime lane mask; C = 0 takes
// it from n at run time.  GOUT: out points to global memory (never LDS).
template <int S, int C = 0, bool GOUT = false>
__device__ __forceinline__ void gen_mc_bits(uint64_t seed, uint64_t key, int n, int n1, uint2* list,
                                            uint32_t* out) {
    static_assert(C >= 0 && C <= S, "chunk count within the bitmask layout");
    const int lane = lane_id();
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    const uint32_t blo = (uint32_t)key, bhi = (uint32_t)(key >> 32);
    const int chunks = C > 0 ? C : (n + kUnitsPerChunk - 1) / kUnitsPerChunk;
    uint32_t u[S][4];
    uint64_t vm[S][4];   // lanes holding a unit < n (wave-uniform)
    if constexpr (C > 0) {
        // all C blocks advance round by round: C independent multiply chains per lane
#pragma unroll
        for (int s = 0; s < S; ++s) {
            u[s][0] = 64u * s + lane;
            u[s][1] = 0u;
            u[s][2] = blo;
            u[s][3] = bhi;
        }
        uint32_t ka = k0, kb = k1;
#pragma unroll
        for (int r = 0; r < 10; ++r) {
#pragma unroll
            for (int s = 0; s < C; ++s) philox_round(u[s][0], u[s][1], u[s][2], u[s][3], ka, kb);
            ka += kPhiloxW0;
            kb += kPhiloxW1;
        }
#pragma unroll
        for (int s = C; s < S; ++s) u[s][0] = u[s][1] = u[s][2] = u[s][3] = 0u;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
        if constexpr (C == 0) {
            if (s < chunks) {
                uint32_t c0 = 64u * s + lane, c1 = 0, c2 = blo, c3 = bhi;
                philox_block(c0, c1, c2, c3, k0, k1);
                u[s][0] = c0; u[s][1] = c1; u[s][2] = c2; u[s][3] = c3;
            } else {
                u[s][0] = u[s][1] = u[s][2] = u[s][3] = 0u;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int left = n - 256 * s - 64 * r;
            if (C > 0 && s < C - 1)
                vm[s][r] = ~0ull;                        // a full chunk
            else if (C > 0 && s >= C)
                vm[s][r] = 0ull;                         // past the last chunk
            else
                vm[s][r] = left >= 64 ? ~0ull : (left <= 0 ? 0ull : ((1ull << left) - 1));
        }
    }
    auto count_below = [&](uint32_t pv) -> int {   // #{valid u < pv}
        int c = 0;
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (s < chunks) c += __builtin_popcountll(ballot(u[s][r] < pv) & vm[s][r]);
        return c;
    };

    // Bracket [lo, hi] (inclusive, 32-bit) around the n1-th smallest value u*:
    // #{u < lo} = clo < n1 <= chi = #{u <= hi}.  A pivot p in (lo, hi] with c = #{u < p}
    // moves lo to p (c < n1) or hi to p - 1 (c >= n1).
    uint32_t lo = 0u, hi = 0xFFFFFFFFu;
    int clo = 0, chi = n;
    if constexpr (S <= 8) {
        // A 256-bin histogram of the keys' top byte (the 1 KB list as LDS counters) gives the
        // first bracket, [b * 2^24, (b + 1) * 2^24 - 1] with b the first bin whose running
        // count reaches n1, in one counting pass; with uniform keys it holds about n / 256
        // values, so the count loop below has little or nothing left to do.
        uint32_t* h = reinterpret_cast<uint32_t*>(list);
        list[2 * lane] = make_uint2(0u, 0u);
        list[2 * lane + 1] = make_uint2(0u, 0u);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (s < chunks && ((vm[s][r] >> lane) & 1ull)) atomicAdd(&h[u[s][r] >> 24], 1u);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const uint2 ha = list[2 * lane], hb = list[2 * lane + 1];   // bins 4 lane .. 4 lane + 3
        const uint32_t c1 = ha.x, c2 = c1 + ha.y, c3 = c2 + hb.x, c4 = c3 + hb.y;
        const uint32_t incl = wave_incl_scan_rows(c4);             // values in bins < 4 lane + 4
        const uint32_t excl = incl - c4;
        // L: the lane holding bin b (wave-uniform); only its values below are read, the other
        // lanes' (need may wrap there) are discarded
        const int L = (int)__builtin_ctzll(ballot(incl >= (uint32_t)n1));
        const uint32_t need = (uint32_t)n1 - excl;                  // >= 1 in lane L
        const uint32_t k = need <= c1 ? 0u : (need <= c2 ? 1u : (need <= c3 ? 2u : 3u));
        const uint32_t before = k == 0u ? 0u : (k == 1u ? c1 : (k == 2u ? c2 : c3));
        const uint32_t upto = k == 0u ? c1 : (k == 1u ? c2 : (k == 2u ? c3 : c4));
        const uint32_t b = 4u * (uint32_t)L + __builtin_amdgcn_readlane(k, L);
        lo = b << 24;
        hi = lo | 0xFFFFFFu;
        clo = (int)__builtin_amdgcn_readlane(excl + before, L);
        chi = (int)__builtin_amdgcn_readlane(excl + upto, L);
        __builtin_amdgcn_wave_barrier();
    }
    // stop at <= 8 bracket values after a few cheap counts, at <= 64 after many; after the
    // histogram bracket (n <= 2048), at <= 64 at once: ranking a few more values in LDS is
    // cheaper than another count pass over 4 S keys per lane
    for (int it = 0; (chi - clo > 64 || (S > 8 && chi - clo > 8 && it < 6)) && lo < hi; ++it) {
        const uint32_t span = hi - lo;
        uint32_t off;
        if (it < 4) {
            // interpolate: unit keys are uniform, so u* sits near the fraction (n1 - clo) / (chi - clo)
            const float f = (float)(n1 - clo) * __builtin_amdgcn_rcpf((float)(chi - clo));
            off = (uint32_t)fminf(fmaxf(f * (float)span, 0.0f), 4294967040.0f);
        } else {
            off = (span >> 1) + 1u;
        }
        off = __builtin_amdgcn_readfirstlane(off);
        const uint32_t p = off == 0u ? lo + 1u : (off >= span ? hi : lo + off);
        const int c = count_below(p);
        if (c < n1) {
            lo = p;
            clo = c;
        } else {
            hi = p - 1u;
            chi = c;
        }
    }

    uint32_t ustar;
    int take, eq_total;
    if (lo == hi) {
        // the bracket holds one value
        ustar = lo;
        take = n1 - clo;
        eq_total = chi - clo;
    } else {
        // collect the <= 64 bracket values, rank them
        const uint32_t span = hi - lo;
        int base = 0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (s < chunks) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const bool f = (u[s][r] - lo) <= span;   // lo <= u <= hi
                    const uint64_t bm = ballot(f) & vm[s][r];
                    if (bm) {
                        // members go to slots base.., the other lanes to their own spare slot
                        const int pos = ((bm >> lane) & 1ull)
                                            ? base + (int)__builtin_amdgcn_mbcnt_hi(
                                                         (uint32_t)(bm >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u))
                                            : 64 + lane;
                        list[pos] = make_uint2(u[s][r], 0u);
                        base += __builtin_popcountll(bm);
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int cnt = chi - clo;
        const int need = n1 - clo;
        int lt = 0, le = 0;
        const uint32_t mine = lane < cnt ? list[lane].x : 0u;
        for (int t = 0; t < cnt; ++t) {
            const uint32_t v = list[t].x;
            lt += v < mine;
            le += v <= mine;
        }
        const bool is_t = lane < cnt && lt < need && need <= le;
        const uint64_t mt = ballot(is_t);
        const int src = (int)__builtin_ctzll(mt);   // wave-uniform: lane reads, not shuffles
        ustar = __builtin_amdgcn_readlane(mine, src);
        const int lts = __builtin_amdgcn_readlane(lt, src);
        const int les = __builtin_amdgcn_readlane(le, src);
        take = need - lts;
        eq_total = les - lts;
        __builtin_amdgcn_wave_barrier();
    }

    // Index threshold among values equal to ustar (only when some must be left out).
    int istar = 0x7FFFFFFF;
    if (take < eq_total) {
        int left = take;
        bool found = false;
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (!found && s < chunks) {
                    uint64_t bm = ballot(u[s][r] == ustar) & vm[s][r];
                    const int pc = __builtin_popcountll(bm);
                    if (left <= pc) {
                        for (int q = 1; q < left; ++q) bm &= bm - 1;
                        istar = 256 * s + 64 * r + (int)__builtin_ctzll(bm);
                        found = true;
                    } else {
                        left -= pc;
                    }
                }
            }
        }
    }

    // Treated indicator and bitmask words.
#pragma unroll
    for (int s = 0; s < S; ++s) {
        uint32_t w[8];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            uint64_t bm = 0;
            if (s < chunks) {
                if (istar == 0x7FFFFFFF) {
                    bm = ballot(u[s][r] <= ustar) & vm[s][r];
                } else {
                    const int unit = 256 * s + 64 * r + lane;
                    bm = ballot(u[s][r] < ustar || (u[s][r] == ustar && unit <= istar)) & vm[s][r];
                }
            }
            w[2 * r] = (uint32_t)bm;
            w[2 * r + 1] = (uint32_t)(bm >> 32);
        }
        if (lane == 0) {
            // streaming stores: the bitmasks are read once, and should not push the contraction's
            // operand records out of L2
            typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
            if constexpr (GOUT) {
                // out is known to be global memory: a store through a generic pointer (a batched
                // pool's comes from a table) would be a flat store, which also counts against the
                // LDS counter, so that the next draw's LDS reads would wait for it
                typedef __attribute__((address_space(1))) u32x4* gptr_t;
                const gptr_t o = (gptr_t)(out + 8 * s);
                __builtin_nontemporal_store(u32x4{w[0], w[1], w[2], w[3]}, o);
                __builtin_nontemporal_store(u32x4{w[4], w[5], w[6], w[7]}, o + 1);
            } else {
                // out may be LDS (the regeneration, FRT and recheck kernels pass per-wave buffers)
                __builtin_nontemporal_store(u32x4{w[0], w[1], w[2], w[3]}, reinterpret_cast<u32x4*>(out + 8 * s));
                __builtin_nontemporal_store(u32x4{w[4], w[5], w[6], w[7]}, reinterpret_cast<u32x4*>(out + 8 * s) + 1);
            }
        }
    }
}

// gen_mc_bits with the chunk count of n fixed at compile time (S / 2 < chunks <= S).
template <int S, bool GOUT = false>
__device__ __forceinline__ void gen_mc_bits_fixed(uint64_t seed, uint64_t key, int n, int n1, uint2* list,
                                                  uint32_t* out) {
    const int chunks = (n + kUnitsPerChunk - 1) / kUnitsPerChunk;
    if constexpr (S == 1) {
        gen_mc_bits<1, 1, GOUT>(seed, key, n, n1, list, out);
    } else if constexpr (S == 2) {
        gen_mc_bits<2, 2, GOUT>(seed, key, n, n1, list, out);
    } else if constexpr (S == 4) {
        if (chunks == 4) gen_mc_bits<4, 4, GOUT>(seed, key, n, n1, list, out);
        else gen_mc_bits<4, 3, GOUT>(seed, key, n, n1, list, out);
    } else if constexpr (S == 8) {
        switch (chunks) {
            case 8: gen_mc_bits<8, 8, GOUT>(seed, key, n, n1, list, out); break;
            case 7: gen_mc_bits<8, 7, GOUT>(seed, key, n, n1, list, out); break;
            case 6: gen_mc_bits<8, 6, GOUT>(seed, key, n, n1, list, out); break;
            default: gen_mc_bits<8, 5, GOUT>(seed, key, n, n1, list, out); break;
        }
    } else {
        gen_mc_bits<S, 0, GOUT>(seed, key, n, n1, list, out);
    }
}

// ---------------------------------------------------------------------------------------
// Exact enumeration: colex unranking, r = sum_t C(i_t, t).  One lane per draw; n <= 64.
// binom[i * 33 + t] = C(i, t) for i <= 64, t <= 32 (0 where undefined), symmetric use of t.
__device__ __forceinline__ uint64_t colex_unrank_mask(uint64_t r, int n, int n1,
                                                      const uint64_t* binom) {
    // C(i, t) for t > 32 via symmetry C(i, i - t); table holds t <= 32.
    auto C = [&](int i, int t) -> uint64_t {
        if (t < 0 || t > i) return 0;
        int tt = t <= i - t ? t : i - t;
        return binom[i * 33 + tt];
    };
    uint64_t mask = 0;
    int hi = n;
    for (int t = n1; t >= 1; --t) {
        int i = hi - 1;
        while (C(i, t) > r) --i;
        mask |= 1ull << i;
        r -= C(i, t);
        hi = i;
    }
    return mask;
}

}  // namespace rr
