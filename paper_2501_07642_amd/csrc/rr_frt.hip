// rr_rand_test: randomization test conditioned on acceptance (section 2.3
// randomization_test; section 4 "Design-based inference"), exact in integers.
//
// Sharp null H0(tau0): Y_i(1) - Y_i(0) = tau0.  The control outcomes are Y - tau0 w_o and
// the statistic of accepted draw k is T_k(tau0) = DiM(w_k, Y - tau0 w_o); the p-value is
// #{k : |T_k| >= |T_o|} / K.
//
// Exactness.  Y is put on the grid 2^-s: Yq_i = rint(Y_i 2^s), s = 61 - t - e (n^2 <= 2^t,
// max|Y| = f 2^e), so every sum below fits its integer type.  With A_k the treated sum of Yq,
// B_k = |T_k and T_o| and tau' = tau0 2^s,
//     n1 n0 T_k = (n A_k - n1 sum Yq) - tau' (n B_k - n1^2) = alpha_k - tau' beta_k.
// A double tau0 is m 2^-E with m odd, so tau' = m 2^D, D = s - E, and the comparison
// |alpha_k - m 2^D beta_k| >= |alpha_o - m 2^D beta_o| (both sides times 2^-D when D < 0)
// is carried out in 128-bit integers.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "rr_internal.h"

namespace rr {

__global__ __launch_bounds__(256) void frt_quantize_kernel(const double* Y, int n, int64_t* Yq, int64_t* meta) {
    // meta[0] = s, meta[1] = sum Yq, meta[2] = 0
    __shared__ double smax[256];
    __shared__ long long ssum[256];
    __shared__ int s_shift;
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, fabs(Y[i]));
    smax[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int sh = 0;
        if (smax[0] > 0.0) {
            int e = 0;
            frexp(smax[0], &e);
            const uint64_t nn = (uint64_t)n * (uint64_t)n - 1;
            const int t = nn == 0 ? 0 : 64 - __builtin_clzll(nn);
            sh = 61 - t - e;
        }
        s_shift = sh;
        meta[0] = sh;
        meta[2] = 0;   // range flag of the null values (set by frt_tau_kernel)
    }
    __syncthreads();
    long long acc = 0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const long long q = (long long)rint(ldexp(Y[i], s_shift));
        Yq[i] = q;
        acc += q;
    }
    ssum[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) ssum[threadIdx.x] += ssum[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) meta[1] = ssum[0];
}

// Per accepted draw: A_k and B_k from the regenerated bitmask (one wave per draw); then
// alpha_k, beta_k.  obs_bits must hold the observed draw's bitmask.
template <int S, bool EXACT>
__global__ __launch_bounds__(256) void frt_stats_kernel(const uint64_t* keys, uint64_t K, uint64_t seed, int n,
                                                        int n1, const uint64_t* binom, const int64_t* Yq,
                                                        const int64_t* meta, const uint32_t* obs_bits,
                                                        int64_t* alpha, int64_t* beta, uint32_t* out_bits) {
    __shared__ uint32_t sbits[4][8 * kMaxS];
    __shared__ uint2 slist[4][128];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const int nw = (n + 31) / 32;
    for (uint64_t k = (uint64_t)blockIdx.x * 4 + wave; k < K; k += (uint64_t)gridDim.x * 4) {
        if constexpr (EXACT) {
            if (lane == 0) {
                const uint64_t m = colex_unrank_mask(keys[k], n, n1, binom);
                sbits[wave][0] = (uint32_t)m;
                sbits[wave][1] = (uint32_t)(m >> 32);
            }
        } else {
            gen_mc_bits_fixed<S>(seed, keys[k], n, n1, slist[wave], sbits[wave]);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        long long a = 0;
        for (int i = lane; i < n; i += 64)
            if ((sbits[wave][i >> 5] >> (i & 31)) & 1u) a += Yq[i];
        a = wave_sum<long long>(a);
        int b = 0;
        if (obs_bits)
            for (int w = lane; w < nw; w += 64) b += __builtin_popcount(sbits[wave][w] & obs_bits[w]);
        b = wave_sum<int>(b);
        if (lane == 0) {
            if (alpha) {
                alpha[k] = (int64_t)n * a - (int64_t)n1 * meta[1];
                beta[k] = (int64_t)n * b - (int64_t)n1 * n1;
            }
        }
        if (out_bits)
            for (int w = lane; w < nw; w += 64) out_bits[w] = sbits[wave][w];
        __builtin_amdgcn_wave_barrier();
    }
}

__device__ __forceinline__ __int128 abs128(__int128 x) { return x < 0 ? -x : x; }

__device__ __forceinline__ int bitlen_dev(unsigned __int128 x) {
    const uint64_t hi = (uint64_t)(x >> 64), lo = (uint64_t)x;
    return hi ? 128 - __builtin_clzll(hi) : (lo ? 64 - __builtin_clzll(lo) : 0);
}

// Per null value g: tau0 = m 2^-E with m odd (m = 0 for tau0 = 0), D = s - E, and the range
// check of the 128-bit comparison (|alpha| <= 2^62, |beta| <= n^2 / 4 + 1); a value outside
// it sets meta[2], and then the count kernel writes nothing.
__global__ void frt_tau_kernel(const double* tau, int64_t G, int n, int64_t* meta, int64_t* tm, int* tD) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const int s = (int)meta[0];
    const double t = tau[g];
    int64_t m = 0;
    int D = 0;
    if (t != 0.0) {
        int e = 0;
        const double f = frexp(t, &e);                    // t = f 2^e, |f| in [0.5, 1)
        int64_t mant = (int64_t)ldexp(f, 53);             // exact: t = mant 2^(e - 53)
        const int tz = __builtin_ctzll((uint64_t)(mant < 0 ? -mant : mant));
        m = mant / ((int64_t)1 << tz);
        D = s - (53 - e - tz);
    }
    const int bbits = bitlen_dev((unsigned __int128)((uint64_t)n * (uint64_t)n / 4 + 1));
    const int mbits = bitlen_dev((unsigned __int128)(uint64_t)(m < 0 ? -m : m));
    const bool ok = D >= 0 ? (mbits + D + bbits <= 125) : (62 - D <= 125 && mbits + bbits <= 125);
    if (!ok) atomicOr((unsigned long long*)&meta[2], 1ull);
    tm[g] = m;
    tD[g] = D;
}

// One workgroup per null value g: counts |alpha_k - tau' beta_k| >= |alpha_o - tau' beta_o|.
__global__ __launch_bounds__(256) void frt_count_kernel(const int64_t* alpha, const int64_t* beta, uint64_t K,
                                                        uint64_t obs, const int64_t* tm, const int* tD,
                                                        const int64_t* meta, uint64_t* counts) {
    __shared__ unsigned long long red[256];
    if (meta[2]) return;   // a null value out of range: the call fails and writes no counts
    const int g = blockIdx.x;
    const __int128 m = tm[g];
    const int D = tD[g];
    auto val = [&](uint64_t k) -> __int128 {
        const __int128 a = alpha[k], b = beta[k];
        if (D >= 0) return a - m * b * ((__int128)1 << D);
        return a * ((__int128)1 << (-D)) - m * b;
    };
    const __int128 vo = abs128(val(obs));
    unsigned long long c = 0;
    for (uint64_t k = threadIdx.x; k < K; k += 256) c += abs128(val(k)) >= vo;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[g] = red[0];
}

template <bool EXACT>
static hipError_t launch_stats(int S, dim3 grid, hipStream_t st, const uint64_t* keys, uint64_t K, uint64_t seed,
                               int n, int n1, const uint64_t* binom, const int64_t* Yq, const int64_t* meta,
                               const uint32_t* obs_bits, int64_t* alpha, int64_t* beta, uint32_t* out_bits) {
#define RR_ST(SV)                                                                                             \
    hipLaunchKernelGGL((frt_stats_kernel<SV, EXACT>), grid, dim3(256), 0, st, keys, K, seed, n, n1, binom, Yq, \
                       meta, obs_bits, alpha, beta, out_bits)
    if (EXACT) {
        RR_ST(1);
    } else {
        switch (S) {
            case 1: RR_ST(1); break;
            case 2: RR_ST(2); break;
            case 4: RR_ST(4); break;
            case 8: RR_ST(8); break;
            case 16: RR_ST(16); break;
            default: return hipErrorInvalidValue;
        }
    }
#undef RR_ST
    return hipGetLastError();
}

const uint64_t* binom_table_ext(int dev);

// Scratch of one randomization test, carved from one device buffer (256-byte aligned parts):
// meta (s, sum Yq, range flag), Yq (n), the observed bitmask (ceil(n / 32) words), alpha and
// beta (K each), the null values and their (m, D) decompositions (G each).
struct FrtScratch {
    int64_t* meta;
    int64_t* Yq;
    uint32_t* obits;
    int64_t* alpha;
    int64_t* beta;
    double* tau;
    int64_t* tm;
    int* tD;
};

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t frt_scratch_bytes(int64_t n, uint64_t K, int64_t G) {
    const size_t g = (size_t)std::max<int64_t>(G, 1);
    return a256(4 * 8) + a256(8 * (size_t)n) + a256(4 * (size_t)((n + 31) / 32)) + 2 * a256(8 * (size_t)K) +
           2 * a256(8 * g) + a256(4 * g);
}

static FrtScratch frt_carve(void* base, int64_t n, uint64_t K, int64_t G) {
    char* b = (char*)base;
    const size_t g = (size_t)std::max<int64_t>(G, 1);
    FrtScratch f;
    f.meta = (int64_t*)b;
    b += a256(4 * 8);
    f.Yq = (int64_t*)b;
    b += a256(8 * (size_t)n);
    f.obits = (uint32_t*)b;
    b += a256(4 * (size_t)((n + 31) / 32));
    f.alpha = (int64_t*)b;
    b += a256(8 * (size_t)K);
    f.beta = (int64_t*)b;
    b += a256(8 * (size_t)K);
    f.tau = (double*)b;
    b += a256(8 * g);
    f.tm = (int64_t*)b;
    b += a256(8 * g);
    f.tD = (int*)b;
    return f;
}

// Argument checks shared by the entry points (host, no device work).
rr_status frt_check(rr_problem* p, int exact, const uint64_t* d_keys, uint64_t K, uint64_t obs_index,
                    const double* d_Y, const double* h_tau0, int64_t G, uint64_t* d_counts, const char* who) {
    if (!p || !d_keys || !d_Y || K == 0 || G < 0 || (G > 0 && (!h_tau0 || !d_counts))) {
        set_error(std::string(who) + ": invalid argument");
        return RR_E_ARG;
    }
    if (obs_index >= K) {
        set_error(std::string(who) + ": observed index not among the accepted keys");
        return RR_E_OBS;
    }
    if (exact && p->P.n > RR_MAX_N_EXACT) {
        set_error(std::string(who) + ": exact keys need n <= 64");
        return RR_E_RANGE;
    }
    for (int64_t g = 0; g < G; ++g)
        if (!std::isfinite(h_tau0[g])) {
            set_error(std::string(who) + ": tau0 must be finite");
            return RR_E_ARG;
        }
    return RR_OK;
}

// The test on a caller-provided scratch buffer of frt_scratch_bytes(n, K, G) bytes: kernels on
// `st`, one synchronisation at the end (for the range flag and tau_hat).  No allocation.
rr_status frt_run(Problem& P, uint64_t seed, int exact, const uint64_t* d_keys, uint64_t K, uint64_t obs_index,
                  const double* d_Y, const double* h_tau0, int64_t G, uint64_t* d_counts, double* h_tau_hat,
                  hipStream_t st, void* scratch, const char* who) {
    const int n = (int)P.n, n1 = (int)P.n1;
    const uint64_t* binom = exact ? binom_table_ext(P.device) : nullptr;
    const FrtScratch f = frt_carve(scratch, P.n, K, G);
#define RR_FHIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            set_error(std::string(who) + ": " + #call + ": " + hipGetErrorString(e_));         \
            return RR_E_DEVICE;                                                                \
        }                                                                                      \
    } while (0)
    hipLaunchKernelGGL(frt_quantize_kernel, dim3(1), dim3(256), 0, st, d_Y, n, f.Yq, f.meta);
    RR_FHIP(hipGetLastError());
    // the observed draw's bitmask
    const uint64_t* okey = d_keys + obs_index;
    if (exact)
        RR_FHIP(launch_stats<true>(P.S, dim3(1), st, okey, 1, seed, n, n1, binom, f.Yq, f.meta, nullptr, nullptr,
                                   nullptr, f.obits));
    else
        RR_FHIP(launch_stats<false>(P.S, dim3(1), st, okey, 1, seed, n, n1, binom, f.Yq, f.meta, nullptr, nullptr,
                                    nullptr, f.obits));
    const dim3 grid((unsigned)std::min<uint64_t>((K + 3) / 4, 4096));
    if (exact)
        RR_FHIP(launch_stats<true>(P.S, grid, st, d_keys, K, seed, n, n1, binom, f.Yq, f.meta, f.obits, f.alpha,
                                   f.beta, nullptr));
    else
        RR_FHIP(launch_stats<false>(P.S, grid, st, d_keys, K, seed, n, n1, binom, f.Yq, f.meta, f.obits, f.alpha,
                                    f.beta, nullptr));
    if (G > 0) {
        RR_FHIP(hipMemcpyAsync(f.tau, h_tau0, sizeof(double) * G, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(frt_tau_kernel, dim3((unsigned)((G + 255) / 256)), dim3(256), 0, st, f.tau, G, n, f.meta,
                           f.tm, f.tD);
        RR_FHIP(hipGetLastError());
        hipLaunchKernelGGL(frt_count_kernel, dim3((unsigned)G), dim3(256), 0, st, f.alpha, f.beta, K, obs_index, f.tm,
                           f.tD, f.meta, d_counts);
        RR_FHIP(hipGetLastError());
    }
    int64_t hmeta[3] = {0, 0, 0};
    int64_t halpha_o = 0;
    RR_FHIP(hipMemcpyAsync(hmeta, f.meta, sizeof(hmeta), hipMemcpyDeviceToHost, st));
    RR_FHIP(hipMemcpyAsync(&halpha_o, f.alpha + obs_index, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    RR_FHIP(hipStreamSynchronize(st));
#undef RR_FHIP
    if (hmeta[2]) {
        set_error(std::string(who) + ": tau0 outside the exact comparison range");
        return RR_E_RANGE;
    }
    if (h_tau_hat) *h_tau_hat = std::ldexp((double)halpha_o, -(int)hmeta[0]) / ((double)n1 * (double)(n - n1));
    return RR_OK;
}

}  // namespace rr

using namespace rr;

extern "C" rr_status rr_rand_test(rr_problem* p, uint64_t seed, int exact, const uint64_t* d_keys, uint64_t K,
                                  uint64_t obs_index, const double* d_Y, const double* h_tau0, int64_t G,
                                  uint64_t* d_counts, double* h_tau_hat, void* stream) {
    rr_status s = frt_check(p, exact, d_keys, K, obs_index, d_Y, h_tau0, G, d_counts, "rr_rand_test");
    if (s != RR_OK) return s;
    Problem& P = p->P;
    if ((s = ensure_aux(P, frt_scratch_bytes(P.n, K, G))) != RR_OK) return s;
    return frt_run(P, seed, exact, d_keys, K, obs_index, d_Y, h_tau0, G, d_counts, h_tau_hat, (hipStream_t)stream,
                   P.aux, "rr_rand_test");
}

extern "C" rr_status rr_rand_test_interval(rr_problem* p, uint64_t seed, int exact, const uint64_t* d_keys,
                                           uint64_t K, uint64_t obs_index, const double* d_Y, const double* h_tau0,
                                           int64_t G, double alpha, uint64_t* d_counts, double* h_tau_hat,
                                           double* h_interval, int* h_contiguous, void* stream) {
    if (!(alpha > 0.0 && alpha < 1.0) || !h_interval || !h_contiguous || G < 1) {
        set_error("rr_rand_test_interval: invalid argument");
        return RR_E_ARG;
    }
    rr_status s = rr_rand_test(p, seed, exact, d_keys, K, obs_index, d_Y, h_tau0, G, d_counts, h_tau_hat, stream);
    if (s != RR_OK) return s;
    std::vector<uint64_t> c((size_t)G);
    RR_HIP(hipMemcpyAsync(c.data(), d_counts, sizeof(uint64_t) * G, hipMemcpyDeviceToHost, (hipStream_t)stream));
    RR_HIP(hipStreamSynchronize((hipStream_t)stream));
    // grid points whose p-value c_g / K exceeds alpha, in the caller's grid order
    int64_t first = -1, last = -1, kept = 0;
    double lo = NAN, hi = NAN;
    for (int64_t g = 0; g < G; ++g) {
        if ((double)c[g] / (double)K > alpha) {
            if (first < 0) first = g;
            last = g;
            ++kept;
            lo = std::isnan(lo) ? h_tau0[g] : std::min(lo, h_tau0[g]);
            hi = std::isnan(hi) ? h_tau0[g] : std::max(hi, h_tau0[g]);
        }
    }
    h_interval[0] = lo;
    h_interval[1] = hi;
    *h_contiguous = kept == 0 || kept == last - first + 1;
    return RR_OK;
}
