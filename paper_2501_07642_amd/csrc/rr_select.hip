// Acceptance: streaming prefilter, exact selection over FP32 bounds, FP64 recheck of the
// guard band, key-ordered tie rule, sorted key-only output.  Also the C-ABI entry points
// of the draw pipeline.
//
// Acceptance rules (section 2.2; Appendix A part C): threshold, M <= a; q-quantile, the
// k = ceil(q N (1 - 1e-12)) smallest M, values within a relative eps = 1e-10 of the k-th
// smallest ordered by key.
//
// Every draw carries an FP32 value m32 and a rigorous error bound e, so the FP64 value lies
// in [lo, hi] = [m32 - e, m32 + e] (both padded outward).  With T_hi / T_lo the k-th smallest
// hi / lo, the k-th smallest M lies in [T_lo, T_hi]; a draw with hi < T_lo (1 - eps) is
// accepted outright, one with lo > T_hi (1 + eps) is rejected outright, and the rest -- the
// guard band -- are recomputed in FP64 and the rule is applied to those values.  While
// streaming, a draw is kept as a candidate only if lo <= U, U = (1 + eps) x the running
// T_hi, which never discards a draw the final selection could need.
#include <algorithm>
#include <cstddef>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>

#include "rr_accept.h"
#include "rr_internal.h"

namespace rr {

const uint64_t* binom_table_ext(int dev);
hipError_t launch_regen(int S, bool exact, const uint64_t* keys, uint64_t K, uint64_t seed, int n, int n1,
                        const uint64_t* binom, uint32_t* out, int nw, int grid, hipStream_t st);

// ---------------------------------------------------------------------------------------
// Error state and timing.
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

struct Timing {
    double total_ms = 0, contract_ms = 0, gen_ms = 0;
    int64_t launches = 0;
    uint64_t band = 0;
};
static thread_local Timing g_timing;
void set_timing(double total_ms, double contract_ms, double gen_ms, int64_t launches, uint64_t band) {
    g_timing.total_ms = total_ms;
    g_timing.contract_ms = contract_ms;
    g_timing.gen_ms = gen_ms;
    g_timing.launches = launches;
    g_timing.band = band;
}

// ---------------------------------------------------------------------------------------
// Device control block.
struct Ctl {
    uint32_t cand_count;
    uint32_t overflow;
    float U;
    uint32_t sel_prefix[2];
    uint32_t sel_krem[2];
    uint32_t sel_fail;
    AcceptState ac;
    uint32_t hist[2][256];
};

// ---------------------------------------------------------------------------------------
// Binomial table for colex unranking (per device, created once).
static std::mutex g_binom_mu;
static uint64_t* g_binom_tab[64] = {};

// The device's table if it was created, else null (never allocates).
const uint64_t* binom_table_ready(int dev) {
    std::lock_guard<std::mutex> g(g_binom_mu);
    return dev >= 0 && dev < 64 ? g_binom_tab[dev] : nullptr;
}

const uint64_t* binom_table(int dev) {
    std::lock_guard<std::mutex> g(g_binom_mu);
    uint64_t** tab = g_binom_tab;
    if (dev < 0 || dev >= 64) return nullptr;
    if (!tab[dev]) {
        std::vector<uint64_t> h(65 * 33, 0);
        for (int i = 0; i <= 64; ++i) {
            uint64_t c = 1;
            for (int t = 0; t <= 32 && t <= i; ++t) {
                h[i * 33 + t] = c;
                // C(i, t+1) = C(i, t) * (i - t) / (t + 1), exact in 128-bit
                c = (uint64_t)((unsigned __int128)c * (uint64_t)(i - t) / (uint64_t)(t + 1));
            }
        }
        uint64_t* p = nullptr;
        if (hipMalloc(&p, h.size() * sizeof(uint64_t)) != hipSuccess) return nullptr;
        if (hipMemcpy(p, h.data(), h.size() * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
        tab[dev] = p;
    }
    return tab[dev];
}

const uint64_t* binom_table_ext(int dev) { return binom_table(dev); }

static bool binom_exact(int64_t n, int64_t k, uint64_t* out) {
    unsigned __int128 c = 1;
    for (int64_t t = 0; t < k; ++t) {
        c = c * (unsigned __int128)(n - t) / (unsigned __int128)(t + 1);
        if (c > ((unsigned __int128)1 << 64) - 1) return false;
    }
    *out = (uint64_t)c;
    return true;
}

// ---------------------------------------------------------------------------------------
// Kernels: radix selection of the k-th smallest of two float arrays (bit patterns of
// non-negative floats order like the values), one 8-bit digit per pass.
__global__ void sel_hist_kernel(const float* a0, const float* a1, const uint32_t* count, uint32_t cap, Ctl* ctl,
                                int shift) {
    __shared__ uint32_t h[2][256];
    for (int i = threadIdx.x; i < 512; i += blockDim.x) (&h[0][0])[i] = 0;
    __syncthreads();
    const uint32_t n = min(*count, cap);   // appends past the capacity were not stored
    const uint32_t m = shift == 24 ? 0u : (0xFFFFFFFFu << (shift + 8));
    const uint32_t p0 = ctl->sel_prefix[0] & m, p1 = ctl->sel_prefix[1] & m;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t x0 = __float_as_uint(a0[i]);
        const uint32_t x1 = __float_as_uint(a1[i]);
        if ((x0 & m) == p0) atomicAdd(&h[0][(x0 >> shift) & 255u], 1u);
        if ((x1 & m) == p1) atomicAdd(&h[1][(x1 >> shift) & 255u], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 512; i += blockDim.x) {
        const uint32_t v = (&h[0][0])[i];
        if (v) atomicAdd(&ctl->hist[0][0] + i, v);
    }
}

__global__ void sel_scan_kernel(Ctl* ctl, int shift) {
    // one wave per selection
    const int s = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t need = ctl->sel_krem[s];
    uint32_t bin, below;
    const bool ok = wave_digit_select(ctl->hist[s], need, &bin, &below);
    if (lane == 0) {
        if (!ok) {
            ctl->sel_fail = 1;
        } else {
            ctl->sel_prefix[s] |= bin << shift;
            ctl->sel_krem[s] = need - below;
        }
    }
    reinterpret_cast<uint4*>(ctl->hist[s])[lane] = make_uint4(0, 0, 0, 0);
}

__global__ void sel_init_kernel(Ctl* ctl) {
    ctl->sel_prefix[0] = ctl->sel_prefix[1] = 0;
    ctl->sel_krem[0] = ctl->sel_krem[1] = ctl->ac.k;
}

__device__ __forceinline__ float f32_up(double x) {
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    return f;
}

__global__ void update_U_kernel(Ctl* ctl) {
    const double thi = (double)__uint_as_float(ctl->sel_prefix[0]);
    const float u = f32_up(thi * (1.0 + kEpsTie));
    ctl->U = fminf(ctl->U, u);
}

// Outright acceptances go to the accepted list; guard-band members to the band list.
__global__ void classify_kernel(const uint64_t* ck, const float* chi, const float* clo, const float* cm,
                                Ctl* ctl, int mode, double a, uint64_t* acc_key, double* acc_m,
                                uint8_t* acc_flag, uint32_t acc_cap, uint64_t* band_key,
                                uint32_t band_cap, uint32_t cand_cap) {
    const uint32_t n = min(ctl->cand_count, cand_cap);
    double lo_cut = 0.0, hi_cut = 0.0;
    if (mode == RR_MODE_QUANTILE) {
        lo_cut = (double)__uint_as_float(ctl->sel_prefix[1]) * (1.0 - kEpsTie);
        hi_cut = (double)__uint_as_float(ctl->sel_prefix[0]) * (1.0 + kEpsTie);
    }
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        bool acc, band;
        classify_one(chi[i], clo[i], mode, a, lo_cut, hi_cut, &acc, &band);
        if (acc) {
            const uint32_t p = atomicAdd(&ctl->ac.acc_count, 1u);
            atomicAdd(&ctl->ac.nL, 1u);
            if (p < acc_cap) {
                acc_key[p] = ck[i];
                acc_m[p] = (double)cm[i];
                acc_flag[p] = 0;
            }
        } else if (band) {
            const uint32_t p = atomicAdd(&ctl->ac.band_count, 1u);
            if (p < band_cap) band_key[p] = ck[i];
        }
    }
}

// flag[i] = 1 for i < min(*count, cap)
__global__ void set_count_kernel(uint32_t* c, uint32_t v) { *c = v; }
__global__ void set_count64_kernel(uint64_t* c, uint64_t v) { *c = v; }

// The control block of a call: zeroed, then the accepted count k and the prefilter bound U
// (a kernel rather than a memset and a host copy, so that a call only enqueues kernels).
__global__ __launch_bounds__(256) void init_ctl_kernel(Ctl* ctl, uint32_t k, float U) {
    uint32_t* words = reinterpret_cast<uint32_t*>(ctl);
    for (uint32_t i = threadIdx.x; i < sizeof(Ctl) / sizeof(uint32_t); i += blockDim.x) words[i] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        ctl->ac.k = k;
        ctl->U = U;
    }
}

// Status and count of an asynchronous call, decided on the device from the control block:
// the same checks the synchronous call makes on the host, in the same order.
__global__ void async_status_kernel(const Ctl* ctl, uint32_t cand_cap, uint64_t capacity, int quantile, uint32_t k,
                                    uint64_t* d_count, int32_t* d_status) {
    int32_t st = RR_OK;
    const uint64_t K = ctl->ac.acc_count;
    if (ctl->cand_count > cand_cap) st = RR_E_UNSUPPORTED;
    else if (ctl->sel_fail || ctl->ac.guard_fail) st = RR_E_DEVICE;
    else if (ctl->overflow) st = RR_E_UNSUPPORTED;
    else if (K > capacity) st = RR_E_CAPACITY;
    else if (quantile && K != k) st = RR_E_DEVICE;
    // RR_E_CAPACITY reports the required count; other errors write no count
    if (st == RR_OK || st == RR_E_CAPACITY) *d_count = K;
    *d_status = st;
}

__global__ void fill_flags_kernel(uint8_t* flag, const uint32_t* count, uint32_t cap) {
    const uint32_t n = min(*count, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) flag[i] = 1;
}

__global__ void cap_band_kernel(Ctl* ctl, uint32_t cap) {
    if (ctl->ac.band_count > cap) {
        ctl->overflow = 1;
        ctl->ac.band_count = cap;
    }
}

// Single-workgroup final acceptance among the guard band.
__global__ __launch_bounds__(1024) void band_accept_kernel(const uint64_t* bkey, const double* bm, uint8_t* work,
                                                           Ctl* ctl, int mode, double a, uint64_t* acc_key,
                                                           double* acc_m, uint8_t* acc_flag, uint32_t acc_cap) {
    __shared__ uint32_t hist[256];
    band_accept_block(bkey, bm, work, &ctl->ac, mode, a, acc_key, acc_m, acc_flag, acc_cap, hist);
}

// ---------------------------------------------------------------------------------------
// Sorting (key, payload index) pairs by key: bitonic sort of 2048-element chunks in LDS,
// then merge passes in which every element finds its place by binary search in the
// partner run (keys are distinct).
constexpr int kSortChunk = 2048;

// n_dev (when set) bounds n on the device: a launch sized for n covers a count known only there.
__device__ __forceinline__ uint32_t sort_count(uint32_t n, const uint32_t* n_dev) {
    return n_dev ? min(n, *n_dev) : n;
}

__global__ __launch_bounds__(1024) void sort_chunk_kernel(const uint64_t* key, uint32_t n_max, const uint32_t* n_dev,
                                                          uint64_t* okey, uint32_t* oidx) {
    __shared__ uint64_t sk[kSortChunk];
    __shared__ uint32_t si[kSortChunk];
    const uint32_t n = sort_count(n_max, n_dev);
    const uint32_t base = blockIdx.x * kSortChunk;
    if (base >= n) return;   // workgroup-uniform
    for (int i = threadIdx.x; i < kSortChunk; i += blockDim.x) {
        const uint32_t g = base + i;
        sk[i] = g < n ? key[g] : ~0ull;
        si[i] = g < n ? g : 0xFFFFFFFFu;
    }
    __syncthreads();
    bitonic_sort_lds<kSortChunk>(sk, si);
    for (int i = threadIdx.x; i < kSortChunk; i += blockDim.x) {
        const uint32_t g = base + i;
        if (g < n) {
            okey[g] = sk[i];
            oidx[g] = si[i];
        }
    }
}

// A pass whose width is at least n copies its input unchanged (every element is in run A and
// run B is empty), so the ping-pong buffer of the result does not depend on the device count.
__global__ void merge_pass_kernel(const uint64_t* ik, const uint32_t* ii, uint32_t n_max, const uint32_t* n_dev,
                                  uint32_t width, uint64_t* ok, uint32_t* oi) {
    const uint32_t n = sort_count(n_max, n_dev);
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const uint32_t pair = g / (2 * width);
    const uint32_t a0 = pair * 2 * width;
    const uint32_t b0 = min(a0 + width, n);
    const uint32_t b1 = min(a0 + 2 * width, n);
    const uint64_t x = ik[g];
    uint32_t pos;
    if (g < b0) {
        // count of B elements < x
        uint32_t lo = b0, hi = b1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (ik[mid] < x) lo = mid + 1; else hi = mid;
        }
        pos = a0 + (g - a0) + (lo - b0);
    } else {
        uint32_t lo = a0, hi = b0;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (ik[mid] < x) lo = mid + 1; else hi = mid;
        }
        pos = a0 + (g - b0) + (lo - a0);
    }
    ok[pos] = x;
    oi[pos] = ii[g];
}

// Writes nothing unless the call's status (when given) is RR_OK.
__global__ void gather_out_kernel(const uint64_t* sk, const uint32_t* si, uint32_t n_max, const uint32_t* n_dev,
                                  const int32_t* status, const double* m, const uint8_t* f, uint64_t* okey,
                                  double* om, uint8_t* of) {
    const uint32_t n = sort_count(n_max, n_dev);
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n || (status && *status != RR_OK)) return;
    okey[g] = sk[g];
    om[g] = m[si[g]];
    if (of && f) of[g] = f[si[g]];
}

// Accepted (key, M, flag) triples sorted by key into the outputs; sk / si are two scratch
// buffers of n entries each.  With n_dev set, n is an upper bound and the count is read on
// the device (asynchronous calls), and `status` gates the output writes.
hipError_t sort_accepted(const uint64_t* acc_key, const double* acc_m, const uint8_t* acc_flag, uint32_t n,
                         uint64_t* const sk[2], uint32_t* const si[2], uint64_t* out_key, double* out_m,
                         uint8_t* out_flag, hipStream_t st, const uint32_t* n_dev, const int32_t* status) {
    if (n == 0) return hipSuccess;
    const uint32_t chunks = (n + kSortChunk - 1) / kSortChunk;
    hipLaunchKernelGGL(sort_chunk_kernel, dim3(chunks), dim3(1024), 0, st, acc_key, n, n_dev, sk[0], si[0]);
    int cur = 0;
    for (uint32_t width = kSortChunk; width < n; width *= 2) {
        hipLaunchKernelGGL(merge_pass_kernel, dim3((n + 255) / 256), dim3(256), 0, st, sk[cur], si[cur], n, n_dev,
                           width, sk[cur ^ 1], si[cur ^ 1]);
        cur ^= 1;
    }
    hipLaunchKernelGGL(gather_out_kernel, dim3((n + 255) / 256), dim3(256), 0, st, sk[cur], si[cur], n, n_dev, status,
                       acc_m, acc_flag, out_key, out_m, out_flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Workspace.
struct WS {
    Ctl* ctl;
    uint64_t* cand_key;
    float* cand_hi;
    float* cand_lo;
    float* cand_m;
    uint64_t* acc_key;
    double* acc_m;
    uint8_t* acc_flag;
    uint64_t* band_key;
    double* band_m;
    uint8_t* band_work;
    uint64_t* sk[2];
    uint32_t* si[2];
    uint32_t* bits[2];
    uint32_t cand_cap, acc_cap, band_cap;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device memory of a released handle kept for the next handle on the same device: the draw
// pipeline's workspace and the auxiliary workspace.  A caller that prepares a new problem for
// every pool (as one step of the benchmark does) then allocates neither again.  Streams and
// events stay with their handle and are destroyed with it: an event's last record belongs to
// the stream it was recorded on, which the next handle knows nothing about.  One slot per
// device; a newer release replaces what the slot holds (those buffers are freed then), and the
// slot lives until the process ends.
namespace {
struct Parked {
    void* ws = nullptr;
    size_t ws_bytes = 0;
    void* aux = nullptr;
    size_t aux_bytes = 0;
};
std::mutex g_park_mu;
Parked g_parked[64];

void release_parked(Parked& s) {
    if (s.ws) hipFree(s.ws);
    if (s.aux) hipFree(s.aux);
    s = Parked{};
}
}  // namespace

// Takes the parked buffers of the handle's device, if the handle has none of its own.
static void adopt_parked(Problem& P) {
    if (P.device < 0 || P.device >= 64 || P.ws || P.aux) return;
    std::lock_guard<std::mutex> g(g_park_mu);
    Parked& s = g_parked[P.device];
    P.ws = s.ws;
    P.ws_bytes = s.ws_bytes;
    P.aux = s.aux;
    P.aux_bytes = s.aux_bytes;
    s = Parked{};
}

// Parks a released handle's buffers (the device is idle: rr_free synchronised it).
static void park(Problem& P) {
    if (!P.ws && !P.aux) return;   // nothing to keep
    Parked mine{P.ws, P.ws_bytes, P.aux, P.aux_bytes};
    P.ws = P.aux = nullptr;
    if (P.device < 0 || P.device >= 64) {
        release_parked(mine);
        return;
    }
    std::lock_guard<std::mutex> g(g_park_mu);
    release_parked(g_parked[P.device]);
    g_parked[P.device] = mine;
}

static rr_status ensure_ws(Problem& P, uint32_t cand_cap, uint32_t acc_cap, uint32_t band_cap, size_t bits_words, WS* w) {
    adopt_parked(P);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t o_ctl = take(sizeof(Ctl));
    const size_t o_ck = take(8ull * cand_cap), o_chi = take(4ull * cand_cap), o_clo = take(4ull * cand_cap),
                 o_cm = take(4ull * cand_cap);
    const size_t o_ak = take(8ull * acc_cap), o_am = take(8ull * acc_cap), o_af = take(acc_cap);
    const size_t o_bk = take(8ull * band_cap), o_bm = take(8ull * band_cap), o_bw = take(band_cap);
    const size_t o_s0 = take(8ull * acc_cap), o_s1 = take(8ull * acc_cap), o_i0 = take(4ull * acc_cap),
                 o_i1 = take(4ull * acc_cap);
    const size_t o_b0 = take(4ull * bits_words), o_b1 = take(4ull * bits_words);
    if (off > P.ws_bytes) {
        // an asynchronous call on this handle may still be using the old workspace
        if (P.ws) RR_HIP(hipDeviceSynchronize());
        if (P.ws) hipFree(P.ws);
        P.ws = nullptr;
        P.ws_bytes = 0;
        RR_HIP(hipMalloc(&P.ws, off));
        P.ws_bytes = off;
    }
    char* b = (char*)P.ws;
    w->ctl = (Ctl*)(b + o_ctl);
    w->cand_key = (uint64_t*)(b + o_ck);
    w->cand_hi = (float*)(b + o_chi);
    w->cand_lo = (float*)(b + o_clo);
    w->cand_m = (float*)(b + o_cm);
    w->acc_key = (uint64_t*)(b + o_ak);
    w->acc_m = (double*)(b + o_am);
    w->acc_flag = (uint8_t*)(b + o_af);
    w->band_key = (uint64_t*)(b + o_bk);
    w->band_m = (double*)(b + o_bm);
    w->band_work = (uint8_t*)(b + o_bw);
    w->sk[0] = (uint64_t*)(b + o_s0);
    w->sk[1] = (uint64_t*)(b + o_s1);
    w->si[0] = (uint32_t*)(b + o_i0);
    w->si[1] = (uint32_t*)(b + o_i1);
    w->bits[0] = (uint32_t*)(b + o_b0);
    w->bits[1] = (uint32_t*)(b + o_b1);
    w->cand_cap = cand_cap;
    w->acc_cap = acc_cap;
    w->band_cap = band_cap;
    return RR_OK;
}

rr_status ensure_aux(Problem& P, size_t bytes) {
    adopt_parked(P);
    bytes = align256(std::max<size_t>(bytes, 256));
    if (bytes <= P.aux_bytes) return RR_OK;
    if (P.aux) RR_HIP(hipDeviceSynchronize());
    if (P.aux) RR_HIP(hipFree(P.aux));
    P.aux = nullptr;
    P.aux_bytes = 0;
    RR_HIP(hipMalloc(&P.aux, bytes));
    P.aux_bytes = bytes;
    return RR_OK;
}

// ---------------------------------------------------------------------------------------
// Error bound constants of the FP32 contraction.
//
// Rounding model of the gfx950 MFMA, measured with single instructions on chosen operands
// (pinned by the GPU tests): a 32x32x16 BF16 MFMA forms the exact products of each half of
// its K range (8 products), aligns them to the largest one and sums them with the bits below
// 2^-24 of the largest dropped, then adds each half-sum to the accumulator with one
// round-to-nearest-even step; a 32x32x2 FP32 MFMA adds its two products one at a time, one
// rounding step each.  With u = 2^-24 each rounding step errs by at most u |partial sum| <=
// u sum|terms|, and a half's dropped bits by at most 7 x 2^-23 x its largest product (twice the
// measured window, as margin) <= 14 u sum|terms|, so for one output
//   split: |G32 - sum(hi + lo)| <= (gamma(4 ks) + gamma(14)) sum(|hi| + |lo|)
//          (2 MFMA per K step, 2 rounding steps each; each product in one half-sum), and
//          |x - hi - lo| <= 2^-18 |x|;
//   fp32:  K steps start from zero (16 rounding steps inside a step) and are summed on the
//          VALU (ks steps): gamma(16 + ks) sum|x32|, and |x - x32| <= 2^-24 |x|.
// Hence |G32_j - G_j| <= kappa cabs_j with cabs_j = sum_i |X~_ij| >= the treated sum (the
// split and FP32 forms use the tighter per-column bounds e_j below in place of kappa cabs_j).  M32
// errs by at most scale (2 kappa sum_j |G32_j| cabs_j + kappa^2 sum_j cabs_j^2) plus the
// FP32 sum of squares (gamma(depth) M32); the kernel bounds sum_j |G32_j| cabs_j by
// ||G32|| ||cabs|| (Cauchy-Schwarz), and the assembled bound is multiplied by kSafety = 4:
// the rounding model is a measured property of the hardware, not a documented one, so the
// bound keeps a factor of four in hand against a model that is off by a rounding step or two
// per MFMA (the price is a wider guard band, rechecked in FP64).
constexpr double kU = 0x1p-24;
constexpr double kSafety = 4.0;

static double gamma_m(double m) { return m * kU / (1.0 - m * kU); }

// Per-column bounds e_j of |G32_j - G_j|, tighter than kappa cabs_j (the same rounding model):
//   rounding: a step errs by at most u times the partial sum so far, which holds only the units
//     already added, so the rounding part is u' sum_i |x_ij| (steps unit i passes through),
//     u' = u / (1 - m u) with m the chain length (the step-weighted sum from the preparation);
//   dropped bits (BF16): each half-sum loses less than 7 x 2^-23 times its largest product
//     (twice the measured window), summed over the halves (sum of per-half maxima), compounded
//     through the chain;
//   representation: the exact residuals x - hi - lo (x - float(x) for FP32), of which a treated
//     set sums at most all the positive or all the negative ones.
// FP32: 16 rounding steps inside each K step on its own units, plus the VALU running total.
double split_column_bound(const Problem& P, double wsum_j, double halfmax_j, double resid_j) {
    const double m = 4.0 * (double)P.ks;
    const double up = kU / (1.0 - m * kU);
    const double planes = 1.0 + 0x1p-8 + 0x1p-16;   // |hi| + |lo| <= |x| (1 + 2^-8 + 2^-18)
    const double round = up * planes * wsum_j;
    const double dropped = 7.0 * 0x1p-23 * planes * halfmax_j * (1.0 + gamma_m(m));
    return (round + dropped + resid_j * (1.0 + gamma_m(m))) * (1.0 + 1e-9);
}

double fp32_column_bound(const Problem& P, double cabs_j, double wsum_j, double resid_j) {
    const double m = 16.0 + (double)P.ks;
    const double up = kU / (1.0 - m * kU);
    return (up * (1.0 + 0x1p-23) * (16.0 * cabs_j + wsum_j) + resid_j * (1.0 + gamma_m(m))) * (1.0 + 1e-9);
}

Bound bound_constants(const Problem& P, int prec) {
    const double ks = (double)P.ks;
    // The per-column criterion M = scale max_j G_j^2 errs by at most
    // scale max_j (2 |G32_j| eps_j + eps_j^2) <= scale (2 max_j |G32_j| eps_max + eps_max^2) with
    // eps_j the bound of |G32_j - G_j|: the sum form's bound with the 2-norms over the columns
    // (||cabs||, ||e||) replaced by their largest entries.
    const bool mx = P.metric == RR_METRIC_MAX_SMD;
    if (prec == RR_PREC_FIXED_I8) {
        // G32 is s q summed exactly; only the representation error (e_j, from the
        // preparation) and the FP32 squares / scalings / sums (depth below) remain.
        const int cb = draw_cb(prec, P.S);
        const int chunks = (int)((P.ncb + cb - 1) / cb);
        const double depth = 16.0 * cb + 2.0 * chunks + 8.0;
        Bound b;
        b.two_kappa = (float)(2.0 * (1.0 + gamma_m(depth)) * (1.0 + 1e-6));
        b.csq = (float)((mx ? P.qerr_max * P.qerr_max : P.qerr_c2) * 1.01);
        b.cnorm = (float)((mx ? P.qerr_max : std::sqrt(P.qerr_c2)) * (1.0 + 1e-6));
        b.gamma_ss = (float)(gamma_m(depth) * 1.01);
        b.safety = 1.0f;   // no MFMA rounding model involved: the int32 sums are exact
        return b;
    }
    if (prec == RR_PREC_GRAM_BF16) {
        const double kappa = (gamma_m(4.0 * ks) + gamma_m(14.0)) * (1.0 + 0x1p-8 + 0x1p-16) + 1.05 * 0x1p-18;
        // G'_j = sum_{i in T} K_ij errs by at most kappa cabsK_j; M = scale sum_{j in T} G'_j, so
        // |M32 - M| <= scale (kappa sum_{j in T} cabsK_j + gamma(depth) sum_{j in T} |G'32_j|),
        // and sum_{j in T} cabsK_j <= the sum of the n1 largest column sums (gram_ctop).
        const int cb = draw_cb(prec, P.S);
        const int chunks = (int)((P.ncb_gram + cb - 1) / cb);
        const double depth = 16.0 * cb + chunks + 6.0;
        Bound b;
        b.two_kappa = 0.0f;
        b.cnorm = 0.0f;
        b.csq = (float)(kappa * P.gram_ctop * 1.01);
        b.gamma_ss = (float)(gamma_m(depth) * 1.01);
        b.safety = (float)kSafety;
        return b;
    }
    // sum_j e_j^2 (largest e_j^2 for the per-column criterion) of the per-column bounds
    const double e2 = prec == RR_PREC_SPLIT_BF16 ? (mx ? P.esplit_max * P.esplit_max : P.esplit_n2)
                                                 : (mx ? P.ef32_max * P.ef32_max : P.ef32_n2);
    const int cb = draw_cb(prec, P.S);
    const int chunks = (int)((P.ncb + cb - 1) / cb);
    const double depth_ss = 16.0 * cb + chunks + 4.0;
    Bound b;
    b.two_kappa = (float)(2.0 * (1.0 + gamma_m(depth_ss)) * (1.0 + 1e-6));
    b.csq = (float)(e2 * 1.01);
    b.cnorm = (float)(std::sqrt(e2) * (1.0 + 1e-6));
    b.gamma_ss = (float)(gamma_m(depth_ss) * 1.01);
    b.safety = (float)kSafety;
    return b;
}

int device_cus(int dev) {
    static int cached[64] = {};
    if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev];
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (dev >= 0 && dev < 64) cached[dev] = cus;
    return cus;
}

ContractArgs make_contract_args(const Problem& P, int prec, const Bound& b) {
    ContractArgs a{};
    a.op = prec == RR_PREC_SPLIT_BF16 ? P.op_split
         : prec == RR_PREC_FIXED_I8   ? P.op_i8
         : prec == RR_PREC_GRAM_BF16  ? P.op_gram
                                      : P.op_f32;
    a.cabs = P.cabs;
    a.bscale = P.bscale;
    a.n = (int)P.n;
    a.ks = (int)P.ks;
    a.ncb = (int)(prec == RR_PREC_GRAM_BF16 ? P.ncb_gram : P.ncb);
    a.scale = (float)P.scale;
    a.two_kappa = b.two_kappa;
    a.csq = b.csq;
    a.cnorm = b.cnorm;
    a.gamma_ss = b.gamma_ss;
    a.safety = b.safety;
    a.maxmode = P.metric == RR_METRIC_MAX_SMD ? 1 : 0;
    return a;
}

// Per-handle resources of the two-stream pipeline: generation runs on an internal stream
// (default priority) and overlaps the contraction of the previous chunk on the caller's
// stream; events order the double-buffered bitmask chunks.
static rr_status ensure_streams(Problem& P, size_t nevents, hipStream_t st) {
    // The events are recorded on the caller's stream too; a call on another stream gets fresh
    // events, so that none is re-recorded after the caller may have destroyed the stream it was
    // last recorded on.
    if (P.events_stream != st) {
        for (hipEvent_t e : P.events) hipEventDestroy(e);
        P.events.clear();
        P.events_stream = st;
    }
    if (!P.gen_stream) RR_HIP(hipStreamCreateWithFlags(&P.gen_stream, hipStreamNonBlocking));
    while (P.events.size() < nevents) {
        hipEvent_t e;
        RR_HIP(hipEventCreate(&e));
        P.events.push_back(e);
    }
    return RR_OK;
}

static hipError_t run_select(WS& w, hipStream_t st) {
    hipLaunchKernelGGL(sel_init_kernel, dim3(1), dim3(1), 0, st, w.ctl);
    for (int shift = 24; shift >= 0; shift -= 8) {
        hipLaunchKernelGGL(sel_hist_kernel, dim3(512), dim3(256), 0, st, w.cand_hi, w.cand_lo,
                           &w.ctl->cand_count, w.cand_cap, w.ctl, shift);
        hipLaunchKernelGGL(sel_scan_kernel, dim3(1), dim3(128), 0, st, w.ctl, shift);
    }
    return hipGetLastError();
}

// The draw pipeline shared by Monte Carlo and exact enumeration.
rr_status draw_pipeline(Problem& P, bool exact, uint64_t seed, uint64_t key_begin, uint64_t N, int mode,
                        double q_or_a, int prec, uint64_t* d_keys, double* d_M, uint8_t* d_flags,
                        uint64_t capacity, uint64_t* h_count, hipStream_t st, const Tune* tune,
                        uint64_t* d_count, int32_t* d_status) {
    // Asynchronous calls (d_status set) only enqueue: every size the host would otherwise read
    // back is bounded from above, and the checks run on the device into d_status / d_count.
    const bool async = d_status != nullptr;
    auto t_start = std::chrono::steady_clock::now();
    if (mode == RR_MODE_CHI2_QUANTILE) {
        // a fixed threshold from the chi-square approximation of M
        if (!(q_or_a > 0.0 && q_or_a <= 1.0)) {
            set_error("rr_draw: q must be in (0, 1]");
            return RR_E_ARG;
        }
        q_or_a = chi2_quantile_of(q_or_a, (double)P.d);
        mode = RR_MODE_THRESHOLD;
    }
    if (N == 0 || !d_keys || !d_M || (async ? !d_count : !h_count) ||
        (mode != RR_MODE_QUANTILE && mode != RR_MODE_THRESHOLD) || !valid_prec(prec)) {
        set_error("rr_draw: invalid argument");
        return RR_E_ARG;
    }
    if (prec == RR_PREC_GRAM_BF16 && P.metric == RR_METRIC_MAX_SMD) {
        set_error("rr_draw: the Gram form has no per-column sums (RR_METRIC_MAX_SMD)");
        return RR_E_ARG;
    }
    uint64_t k = 0;
    if (mode == RR_MODE_QUANTILE) {
        if (!(q_or_a > 0.0 && q_or_a <= 1.0)) {
            set_error("rr_draw: q must be in (0, 1]");
            return RR_E_ARG;
        }
        k = (uint64_t)std::ceil(q_or_a * (double)N * (1.0 - kQFuzz));
        k = std::min<uint64_t>(std::max<uint64_t>(k, 1), N);
        if (k > capacity) {
            if (async) {
                hipLaunchKernelGGL(set_count64_kernel, dim3(1), dim3(1), 0, st, d_count, k);
                RR_HIP(hipGetLastError());
            } else {
                *h_count = k;
            }
            set_error("rr_draw: capacity below the accepted count");
            return RR_E_CAPACITY;
        }
        if (k > (1u << 24)) {
            set_error("rr_draw: accepted count above 2^24 per call");
            return RR_E_UNSUPPORTED;
        }
    } else if (std::isnan(q_or_a)) {
        set_error("rr_draw: threshold is NaN");
        return RR_E_ARG;
    }
    rr_status s = RR_OK;
    if (prec == RR_PREC_GRAM_BF16 && (s = ensure_gram(P, st)) != RR_OK) return s;
    // The launch configuration is settled before any workspace pointer is taken: a first call
    // of a tuning bucket probes candidates by running this pipeline on the same handle, and
    // those runs may grow (reallocate) the workspace and the event list.
    const Tune tn = tune ? *tune : tune_for(P, prec, exact, N, st, !async);
    // Chunks of draws: the bitmasks of chunk c are generated on the internal stream while chunk
    // c - 1 is contracted on the caller's stream (at least four chunks when N allows).
    const int clog = std::min(21, std::max(16, tn.chunk_log2));
    uint64_t chunk = std::min<uint64_t>(std::max<uint64_t>((N + 3) / 4, 1u << 16), 1ull << clog);
    chunk = std::min<uint64_t>(chunk, N);
    const uint64_t nchunks = (N + chunk - 1) / chunk;
    const size_t wpd = 8ull * P.S;
    const uint32_t cand_cap = (uint32_t)std::max<uint64_t>(chunk + (1u << 20), 1u << 23);
    const uint32_t acc_cap = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(capacity, 1), cand_cap);
    const uint32_t band_cap = 1u << 20;
    WS w;
    if ((s = ensure_ws(P, cand_cap, acc_cap, band_cap, chunk * wpd, &w)) != RR_OK) return s;
    if ((s = ensure_streams(P, 4 * nchunks + 1, st)) != RR_OK) return s;
    const void* const ws_in_use = P.ws;
    const Bound b = bound_constants(P, prec);
    const uint64_t* binom = exact ? binom_table(P.device) : nullptr;
    if (exact && !binom) {
        set_error("rr_draw_exact: binomial table allocation failed");
        return RR_E_DEVICE;
    }

    {
        float U = INFINITY;
        if (mode == RR_MODE_THRESHOLD) {
            U = (float)q_or_a;
            if ((double)U < q_or_a) U = std::nextafter(U, INFINITY);
        }
        hipLaunchKernelGGL(init_ctl_kernel, dim3(1), dim3(256), 0, st, w.ctl, (uint32_t)k, U);
        RR_HIP(hipGetLastError());
    }
    hipEvent_t* ev = P.events.data();
    // per chunk c: contraction start / end (4c, 4c + 1), generation start / end (4c + 2, 4c + 3);
    // the ends also order the two streams: chunk c's contraction waits for its generation, and
    // generation into a bitmask buffer waits for the contraction of the chunk that last used it
    hipEvent_t ev_start = ev[0];
    hipEvent_t* ev_t = ev + 1;
    const int cus = device_cus(P.device);
    GenArgs g{};
    g.seed = seed;
    g.binom = binom;
    g.n = (int)P.n;
    g.n1 = (int)P.n1;
    ContractArgs a = make_contract_args(P, prec, b);
    a.cand_key = w.cand_key;
    a.cand_hi = w.cand_hi;
    a.cand_lo = w.cand_lo;
    a.cand_m = w.cand_m;
    a.cand_count = &w.ctl->cand_count;
    a.cand_cap = cand_cap;
    RR_HIP(hipEventRecord(ev_start, st));
    RR_HIP(hipStreamWaitEvent(P.gen_stream, ev_start, 0));
    for (uint64_t c = 0; c < nchunks; ++c) {
        const int bsel = (int)(c & 1);
        const uint64_t off = c * chunk;
        const uint64_t num = std::min<uint64_t>(N - off, chunk);
        if (c >= 2) RR_HIP(hipStreamWaitEvent(P.gen_stream, ev_t[4 * (c - 2) + 1], 0));
        g.key_begin = key_begin + off;
        g.num = num;
        g.out = w.bits[bsel];
        RR_HIP(hipEventRecord(ev_t[4 * c + 2], P.gen_stream));
        const uint64_t gen_units = exact ? (num + 63) / 64 : num;
        RR_HIP(launch_gen(P.S, exact, g, (int)std::min<uint64_t>((gen_units + 3) / 4, (uint64_t)cus * tn.gen_wg),
                          P.gen_stream));
        RR_HIP(hipEventRecord(ev_t[4 * c + 3], P.gen_stream));
        RR_HIP(hipStreamWaitEvent(st, ev_t[4 * c + 3], 0));
        a.bits = w.bits[bsel];
        a.num = num;
        a.key_begin = key_begin + off;
        a.U = (mode == RR_MODE_QUANTILE && c == 0) ? nullptr : &w.ctl->U;
        const uint64_t tiles = (num + contract_tile(prec, P.S, tn.db) - 1) / contract_tile(prec, P.S, tn.db);
        RR_HIP(hipEventRecord(ev_t[4 * c], st));
        RR_HIP(launch_contract(P.S, prec, tn.db, false, a, (int)std::min<uint64_t>(tiles, (uint64_t)cus), st));
        RR_HIP(hipEventRecord(ev_t[4 * c + 1], st));
        if (mode == RR_MODE_QUANTILE && c + 1 < nchunks && (c == 0 || c % 8 == 7)) {
            RR_HIP(run_select(w, st));
            hipLaunchKernelGGL(update_U_kernel, dim3(1), dim3(1), 0, st, w.ctl);
            RR_HIP(hipGetLastError());
        }
    }
    if (P.ws != ws_in_use) {
        set_error("rr_draw: workspace replaced during the call");
        return RR_E_DEVICE;
    }
    double contract_ms = 0, gen_ms = 0;
    Ctl hc{};
    if (!async) {
        RR_HIP(hipStreamSynchronize(st));
        for (uint64_t c = 0; c < nchunks; ++c) {
            float m1 = 0, m2 = 0;
            RR_HIP(hipEventElapsedTime(&m1, ev_t[4 * c], ev_t[4 * c + 1]));
            RR_HIP(hipEventElapsedTime(&m2, ev_t[4 * c + 2], ev_t[4 * c + 3]));
            contract_ms += m1;
            gen_ms += m2;
        }
        RR_HIP(hipMemcpyAsync(&hc, w.ctl, offsetof(Ctl, hist), hipMemcpyDeviceToHost, st));
        RR_HIP(hipStreamSynchronize(st));
        if (hc.cand_count > cand_cap) {
            set_error("rr_draw: candidate buffer overflow (too many draws near the boundary)");
            return RR_E_UNSUPPORTED;
        }
    }
    const int64_t launches = (int64_t)nchunks;
    // grids: from the candidate count when it is known on the host, else persistent
    const uint32_t nc = async ? cand_cap : hc.cand_count;
    if (mode == RR_MODE_QUANTILE) RR_HIP(run_select(w, st));
    {
        const int grid = (int)std::max<uint32_t>(1, std::min<uint32_t>((nc + 255) / 256, 4096));
        hipLaunchKernelGGL(classify_kernel, dim3(grid), dim3(256), 0, st, w.cand_key, w.cand_hi, w.cand_lo,
                           w.cand_m, w.ctl, mode, q_or_a, w.acc_key, w.acc_m, w.acc_flag, acc_cap, w.band_key,
                           band_cap, cand_cap);
        RR_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(cap_band_kernel, dim3(1), dim3(1), 0, st, w.ctl, band_cap);
    RecheckArgs ra{};
    ra.X64 = P.X64;
    ra.keys = w.band_key;
    ra.count = &w.ctl->ac.band_count;
    ra.cap = band_cap;
    ra.seed = seed;
    ra.binom = binom;
    ra.n = (int)P.n;
    ra.n1 = (int)P.n1;
    ra.d = (int)P.d;
    ra.scale = P.scale;
    ra.maxmode = P.metric == RR_METRIC_MAX_SMD ? 1 : 0;
    ra.out = w.band_m;
    RR_HIP(launch_recheck(P.S, exact, ra, (int)std::min<uint64_t>((nc + 15) / 16 + 1, (uint64_t)cus * 2), st));
    if (refine_accepted(P, prec)) {
        // the draws accepted outright are reported with their FP64 values too
        RecheckArgs rf = ra;
        rf.keys = w.acc_key;
        rf.count = &w.ctl->ac.acc_count;
        rf.cap = acc_cap;
        rf.out = w.acc_m;
        RR_HIP(launch_recheck(P.S, exact, rf, (int)std::min<uint64_t>((std::min<uint64_t>(nc, acc_cap) + 15) / 16 + 1,
                                                                      (uint64_t)cus * 2), st));
        hipLaunchKernelGGL(fill_flags_kernel, dim3(64), dim3(256), 0, st, w.acc_flag, &w.ctl->ac.acc_count, acc_cap);
        RR_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(band_accept_kernel, dim3(1), dim3(1024), 0, st, w.band_key, w.band_m, w.band_work, w.ctl,
                       mode, q_or_a, w.acc_key, w.acc_m, w.acc_flag, acc_cap);
    RR_HIP(hipGetLastError());
    if (async) {
        // status and count on the device; the sort covers the largest count that can be
        // written (k, or the capacity) and reads the actual one there
        hipLaunchKernelGGL(async_status_kernel, dim3(1), dim3(1), 0, st, w.ctl, cand_cap, capacity,
                           mode == RR_MODE_QUANTILE ? 1 : 0, (uint32_t)k, d_count, d_status);
        RR_HIP(hipGetLastError());
        const uint32_t n_max = mode == RR_MODE_QUANTILE ? (uint32_t)k : acc_cap;
        RR_HIP(sort_accepted(w.acc_key, w.acc_m, w.acc_flag, n_max, w.sk, w.si, d_keys, d_M, d_flags, st,
                             &w.ctl->ac.acc_count, d_status));
        return RR_OK;
    }
    RR_HIP(hipMemcpyAsync(&hc, w.ctl, offsetof(Ctl, hist), hipMemcpyDeviceToHost, st));
    RR_HIP(hipStreamSynchronize(st));
    if (hc.sel_fail || hc.ac.guard_fail) {
        set_error("rr_draw: selection failed (guard band inconsistent)");
        return RR_E_DEVICE;
    }
    if (hc.overflow) {
        set_error("rr_draw: guard band larger than the recheck capacity");
        return RR_E_UNSUPPORTED;
    }
    const uint64_t K = hc.ac.acc_count;
    if (K > capacity) {
        *h_count = K;
        set_error("rr_draw: capacity below the accepted count");
        return RR_E_CAPACITY;
    }
    if (mode == RR_MODE_QUANTILE && K != k) {
        set_error("rr_draw: accepted count differs from k");
        return RR_E_DEVICE;
    }
    if (K > 0) {
        RR_HIP(sort_accepted(w.acc_key, w.acc_m, w.acc_flag, (uint32_t)K, w.sk, w.si, d_keys, d_M, d_flags, st));
        RR_HIP(hipStreamSynchronize(st));
    }
    *h_count = K;
    g_timing.contract_ms = contract_ms;
    g_timing.gen_ms = gen_ms;
    g_timing.launches = launches;
    g_timing.band = hc.ac.band_count;
    g_timing.total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return RR_OK;
}

// M32 / error bound / M64 of given draws: generation into `bits` (8 S words per draw), the
// contraction in evaluation mode, and the FP64 recomputation (count from `cnt`).  Enqueues only.
rr_status balance_keys_enqueue(Problem& P, uint64_t seed, bool exact, const uint64_t* binom,
                                      const uint64_t* d_keys, uint64_t K, int precision, float* d_M32,
                                      float* d_err, double* d_M64, uint32_t* cnt, uint32_t* bits,
                                      hipStream_t st) {
    const int cus = device_cus(P.device);
    if (d_M32) {
        const Bound b = bound_constants(P, precision);
        GenArgs g{};
        g.seed = seed;
        g.num = K;
        g.keylist = d_keys;
        g.binom = binom;
        g.n = (int)P.n;
        g.n1 = (int)P.n1;
        g.out = bits;
        const uint64_t gen_units = exact ? (K + 63) / 64 : K;
        hipError_t e = launch_gen(P.S, exact, g, (int)std::min<uint64_t>((gen_units + 3) / 4, (uint64_t)cus * kGenWgPerCu), st);
        ContractArgs a = make_contract_args(P, precision, b);
        a.bits = bits;
        a.num = K;
        a.keylist = d_keys;
        a.out_m32 = d_M32;
        a.out_err = d_err;
        const uint64_t tiles = (K + contract_tile(precision, P.S, 0) - 1) / contract_tile(precision, P.S, 0);
        if (e == hipSuccess) e = launch_contract(P.S, precision, 0, false, a, (int)std::min<uint64_t>(tiles, (uint64_t)cus), st);
        RR_HIP(e);
    }
    if (d_M64) {
        const uint32_t k32 = (uint32_t)K;
        hipLaunchKernelGGL(set_count_kernel, dim3(1), dim3(1), 0, st, cnt, k32);
        RR_HIP(hipGetLastError());
        RecheckArgs ra{};
        ra.X64 = P.X64;
        ra.keys = d_keys;
        ra.count = cnt;
        ra.cap = k32;
        ra.seed = seed;
        ra.binom = binom;
        ra.n = (int)P.n;
        ra.n1 = (int)P.n1;
        ra.d = (int)P.d;
        ra.scale = P.scale;
        ra.maxmode = P.metric == RR_METRIC_MAX_SMD ? 1 : 0;
        ra.out = d_M64;
        RR_HIP(launch_recheck(P.S, exact, ra, (int)std::min<uint64_t>((K + 15) / 16, (uint64_t)cus * 2), st));
    }
    return RR_OK;
}

int pow2_chunks(int n);
rr_status prepare_impl(const void* dX, int x_dtype, int64_t n, int64_t d, int64_t ldx, int64_t n1,
                       double ridge_rel, int metric, hipStream_t st, rr_problem** out);

}  // namespace rr

using namespace rr;

extern "C" {

const char* rr_last_error(void) { return g_err.c_str(); }

rr_status rr_prepare(const void* d_X, int x_dtype, int64_t n, int64_t d, int64_t ldx, int64_t n1,
                     double ridge_rel, void* stream, rr_problem** out) {
    return prepare_impl(d_X, x_dtype, n, d, ldx, n1, ridge_rel, RR_METRIC_MAHALANOBIS, (hipStream_t)stream, out);
}

rr_status rr_prepare_metric(const void* d_X, int x_dtype, int64_t n, int64_t d, int64_t ldx, int64_t n1,
                            double ridge_rel, int metric, void* stream, rr_problem** out) {
    return prepare_impl(d_X, x_dtype, n, d, ldx, n1, ridge_rel, metric, (hipStream_t)stream, out);
}

void rr_free(rr_problem* p) {
    if (!p) return;
    Problem& P = p->P;
    hipDeviceSynchronize();   // asynchronous calls on this handle may still be running
    hipFree(P.mem);   // X64, L, mu, the operand records, bscale, cabs
    hipFree(P.op_gram);
    park(P);   // the workspaces go to the next handle on this device
    for (hipEvent_t e : P.events) hipEventDestroy(e);
    if (P.gen_stream) hipStreamDestroy(P.gen_stream);
    free_batch_state(P);
    delete p;
}

int64_t rr_problem_n(const rr_problem* p) { return p ? p->P.n : 0; }
int64_t rr_problem_d(const rr_problem* p) { return p ? p->P.d : 0; }
int64_t rr_problem_n1(const rr_problem* p) { return p ? p->P.n1 : 0; }
double rr_problem_lambda(const rr_problem* p) { return p ? p->P.lambda : 0.0; }

rr_status rr_draw_balance(rr_problem* p, uint64_t seed, uint64_t key_begin, uint64_t num_draws, int mode,
                          double q_or_a, int precision, uint64_t* d_keys, double* d_M, uint8_t* d_flags,
                          uint64_t capacity, uint64_t* h_count, void* stream) {
    if (!p) {
        set_error("rr_draw_balance: null handle");
        return RR_E_ARG;
    }
    if (key_begin + num_draws < key_begin) {
        set_error("rr_draw_balance: key range wraps");
        return RR_E_ARG;
    }
    return draw_pipeline(p->P, false, seed, key_begin, num_draws, mode, q_or_a, precision, d_keys, d_M, d_flags,
                         capacity, h_count, (hipStream_t)stream, nullptr);
}

rr_status rr_draw_balance_async(rr_problem* p, uint64_t seed, uint64_t key_begin, uint64_t num_draws, int mode,
                                double q_or_a, int precision, uint64_t* d_keys, double* d_M, uint8_t* d_flags,
                                uint64_t capacity, uint64_t* d_count, int32_t* d_status, void* stream) {
    if (!p || !d_status) {
        set_error("rr_draw_balance_async: null handle or status pointer");
        return RR_E_ARG;
    }
    if (key_begin + num_draws < key_begin) {
        set_error("rr_draw_balance_async: key range wraps");
        return RR_E_ARG;
    }
    return draw_pipeline(p->P, false, seed, key_begin, num_draws, mode, q_or_a, precision, d_keys, d_M, d_flags,
                         capacity, nullptr, (hipStream_t)stream, nullptr, d_count, d_status);
}

rr_status rr_draw_exact(rr_problem* p, int mode, double q_or_a, int precision, uint64_t* d_keys, double* d_M,
                        uint8_t* d_flags, uint64_t capacity, uint64_t* h_count, void* stream) {
    if (!p) {
        set_error("rr_draw_exact: null handle");
        return RR_E_ARG;
    }
    uint64_t total = 0;
    if (p->P.n > RR_MAX_N_EXACT || !binom_exact(p->P.n, p->P.n1, &total) || total >= (1ull << 40)) {
        set_error("rr_draw_exact: C(n, n1) too large for enumeration");
        return RR_E_RANGE;
    }
    return draw_pipeline(p->P, true, 0, 0, total, mode, q_or_a, precision, d_keys, d_M, d_flags, capacity, h_count,
                         (hipStream_t)stream, nullptr);
}

rr_status rr_regenerate(rr_problem* p, uint64_t seed, int exact, const uint64_t* d_keys, uint64_t K,
                        uint32_t* d_bits, void* stream) {
    if (!p || (!d_keys && K) || (!d_bits && K)) {
        set_error("rr_regenerate: invalid argument");
        return RR_E_ARG;
    }
    if (K == 0) return RR_OK;
    Problem& P = p->P;
    if (exact && P.n > RR_MAX_N_EXACT) {
        set_error("rr_regenerate: exact keys need n <= 64");
        return RR_E_RANGE;
    }
    const uint64_t* binom = exact ? binom_table(P.device) : nullptr;
    const int nw = (int)((P.n + 31) / 32);
    const int grid = (int)std::min<uint64_t>((K + 3) / 4, (uint64_t)device_cus(P.device) * 8);
    hipStream_t st = (hipStream_t)stream;
    RR_HIP(launch_regen(P.S, exact != 0, d_keys, K, seed, (int)P.n, (int)P.n1, binom, d_bits, nw, grid, st));
    RR_HIP(hipStreamSynchronize(st));
    return RR_OK;
}

rr_status rr_balance_keys(rr_problem* p, uint64_t seed, int exact, const uint64_t* d_keys, uint64_t K,
                          int precision, float* d_M32, float* d_err, double* d_M64, void* stream) {
    if (!p || (K && !d_keys) || !valid_prec(precision) ||
        (!d_M32) != (!d_err) || K > 0xFFFFFFFFull) {
        set_error("rr_balance_keys: invalid argument");
        return RR_E_ARG;
    }
    if (K == 0) return RR_OK;
    Problem& P = p->P;
    if (exact && P.n > RR_MAX_N_EXACT) {
        set_error("rr_balance_keys: exact keys need n <= 64");
        return RR_E_RANGE;
    }
    if (d_M32 && precision == RR_PREC_GRAM_BF16 && P.metric == RR_METRIC_MAX_SMD) {
        set_error("rr_balance_keys: the Gram form has no per-column sums (RR_METRIC_MAX_SMD)");
        return RR_E_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    const uint64_t* binom = exact ? binom_table(P.device) : nullptr;
    if (exact && !binom) {
        set_error("rr_balance_keys: binomial table allocation failed");
        return RR_E_DEVICE;
    }
    // workspace: the count (first 256 bytes), then the bitmasks of the draws
    const rr_status sa = ensure_aux(P, 256 + (d_M32 ? sizeof(uint32_t) * 8 * P.S * K : 0));
    if (sa != RR_OK) return sa;
    if (d_M32 && precision == RR_PREC_GRAM_BF16) {
        const rr_status s = ensure_gram(P, st);
        if (s != RR_OK) return s;
    }
    const rr_status s = balance_keys_enqueue(P, seed, exact != 0, binom, d_keys, K, precision, d_M32, d_err, d_M64,
                                             (uint32_t*)P.aux, (uint32_t*)((char*)P.aux + 256), st);
    if (s != RR_OK) return s;
    RR_HIP(hipStreamSynchronize(st));
    return RR_OK;
}

rr_status rr_last_timing(double* total_ms, double* contract_ms, double* gen_ms, int64_t* draw_launches,
                         uint64_t* band_size) {
    if (total_ms) *total_ms = g_timing.total_ms;
    if (contract_ms) *contract_ms = g_timing.contract_ms;
    if (gen_ms) *gen_ms = g_timing.gen_ms;
    if (draw_launches) *draw_launches = g_timing.launches;
    if (band_size) *band_size = g_timing.band;
    return RR_OK;
}

}  // extern "C"
