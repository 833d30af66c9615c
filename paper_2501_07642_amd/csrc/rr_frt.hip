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
#include <cmath>

#include "rr_internal.h"

namespace rr {

__global__ __launch_bounds__(256) void frt_quantize_kernel(const double* Y, int n, int64_t* Yq, int64_t* meta) {
    // meta[0] = s, meta[1] = sum Yq
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

// One workgroup per null value g: counts |alpha_k - tau' beta_k| >= |alpha_o - tau' beta_o|.
__global__ __launch_bounds__(256) void frt_count_kernel(const int64_t* alpha, const int64_t* beta, uint64_t K,
                                                        uint64_t obs, const int64_t* tm, const int* tD,
                                                        uint64_t* counts) {
    __shared__ unsigned long long red[256];
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

static int bitlen_u(unsigned __int128 x) {
    int b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

const uint64_t* binom_table_ext(int dev);

}  // namespace rr

using namespace rr;

extern "C" rr_status rr_rand_test(rr_problem* p, uint64_t seed, int exact, const uint64_t* d_keys, uint64_t K,
                                  uint64_t obs_index, const double* d_Y, const double* h_tau0, int64_t G,
                                  uint64_t* d_counts, double* h_tau_hat, void* stream) {
    if (!p || !d_keys || !d_Y || K == 0 || G < 0 || (G > 0 && (!h_tau0 || !d_counts))) {
        set_error("rr_rand_test: invalid argument");
        return RR_E_ARG;
    }
    if (obs_index >= K) {
        set_error("rr_rand_test: observed index not among the accepted keys");
        return RR_E_OBS;
    }
    Problem& P = p->P;
    if (exact && P.n > RR_MAX_N_EXACT) {
        set_error("rr_rand_test: exact keys need n <= 64");
        return RR_E_RANGE;
    }
    for (int64_t g = 0; g < G; ++g)
        if (!std::isfinite(h_tau0[g])) {
            set_error("rr_rand_test: tau0 must be finite");
            return RR_E_ARG;
        }
    hipStream_t st = (hipStream_t)stream;
    const int n = (int)P.n, n1 = (int)P.n1;
    const int nw = (n + 31) / 32;
    const uint64_t* binom = exact ? binom_table_ext(P.device) : nullptr;
    int64_t *Yq = nullptr, *meta = nullptr, *alpha = nullptr, *beta = nullptr, *tm = nullptr;
    int* tD = nullptr;
    uint32_t* obits = nullptr;
    uint64_t* okey = nullptr;
    auto cleanup = [&]() {
        hipFree(Yq);
        hipFree(meta);
        hipFree(alpha);
        hipFree(beta);
        hipFree(tm);
        hipFree(tD);
        hipFree(obits);
    };
#define RR_FHIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            set_error(std::string("rr_rand_test: ") + #call + ": " + hipGetErrorString(e_));    \
            cleanup();                                                                         \
            return RR_E_DEVICE;                                                                \
        }                                                                                      \
    } while (0)
    RR_FHIP(hipMalloc(&Yq, sizeof(int64_t) * n));
    RR_FHIP(hipMalloc(&meta, sizeof(int64_t) * 2));
    RR_FHIP(hipMalloc(&alpha, sizeof(int64_t) * K));
    RR_FHIP(hipMalloc(&beta, sizeof(int64_t) * K));
    RR_FHIP(hipMalloc(&obits, sizeof(uint32_t) * nw));
    RR_FHIP(hipMalloc(&tm, sizeof(int64_t) * std::max<int64_t>(G, 1)));
    RR_FHIP(hipMalloc(&tD, sizeof(int) * std::max<int64_t>(G, 1)));
    hipLaunchKernelGGL(frt_quantize_kernel, dim3(1), dim3(256), 0, st, d_Y, n, Yq, meta);
    RR_FHIP(hipGetLastError());
    // observed draw's bitmask
    okey = const_cast<uint64_t*>(d_keys + obs_index);
    if (exact)
        RR_FHIP(launch_stats<true>(P.S, dim3(1), st, okey, 1, seed, n, n1, binom, Yq, meta, nullptr, nullptr,
                                   nullptr, obits));
    else
        RR_FHIP(launch_stats<false>(P.S, dim3(1), st, okey, 1, seed, n, n1, binom, Yq, meta, nullptr, nullptr,
                                    nullptr, obits));
    const dim3 grid((unsigned)std::min<uint64_t>((K + 3) / 4, 4096));
    if (exact)
        RR_FHIP(launch_stats<true>(P.S, grid, st, d_keys, K, seed, n, n1, binom, Yq, meta, obits, alpha, beta,
                                   nullptr));
    else
        RR_FHIP(launch_stats<false>(P.S, grid, st, d_keys, K, seed, n, n1, binom, Yq, meta, obits, alpha, beta,
                                    nullptr));
    int64_t hmeta[2];
    int64_t halpha_o = 0;
    RR_FHIP(hipMemcpyAsync(hmeta, meta, sizeof(hmeta), hipMemcpyDeviceToHost, st));
    RR_FHIP(hipMemcpyAsync(&halpha_o, alpha + obs_index, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    RR_FHIP(hipStreamSynchronize(st));
    const int s = (int)hmeta[0];
    // tau0 = m 2^-E (m odd), D = s - E; range of the 128-bit comparison:
    // |alpha| <= 2^62, |beta| <= n1 n0 <= n^2/4.
    std::vector<int64_t> hm((size_t)std::max<int64_t>(G, 1));
    std::vector<int> hD((size_t)std::max<int64_t>(G, 1));
    const int bbits = bitlen_u((unsigned __int128)((uint64_t)n * (uint64_t)n / 4 + 1));
    for (int64_t g = 0; g < G; ++g) {
        const double t = h_tau0[g];
        int64_t m = 0;
        int D = 0;
        if (t != 0.0) {
            int e = 0;
            const double f = std::frexp(t, &e);              // t = f 2^e, |f| in [0.5, 1)
            int64_t mant = (int64_t)std::ldexp(f, 53);      // exact: t = mant 2^(e-53)
            int E = 53 - e;
            while ((mant & 1) == 0) {
                mant /= 2;
                --E;
            }
            m = mant;
            D = s - E;
        }
        const int mbits = bitlen_u((unsigned __int128)(m < 0 ? -m : m));
        const bool ok = D >= 0 ? (mbits + D + bbits <= 125) : (62 - D <= 125 && mbits + bbits <= 125);
        if (!ok) {
            set_error("rr_rand_test: tau0 outside the exact comparison range");
            cleanup();
            return RR_E_RANGE;
        }
        hm[g] = m;
        hD[g] = D;
    }
    if (G > 0) {
        RR_FHIP(hipMemcpyAsync(tm, hm.data(), sizeof(int64_t) * G, hipMemcpyHostToDevice, st));
        RR_FHIP(hipMemcpyAsync(tD, hD.data(), sizeof(int) * G, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(frt_count_kernel, dim3((unsigned)G), dim3(256), 0, st, alpha, beta, K, obs_index, tm, tD,
                           d_counts);
        RR_FHIP(hipGetLastError());
    }
    RR_FHIP(hipStreamSynchronize(st));
    if (h_tau_hat)
        *h_tau_hat = std::ldexp((double)halpha_o, -s) / ((double)n1 * (double)(n - n1));
    cleanup();
#undef RR_FHIP
    return RR_OK;
}
