// FP64 recomputation of M for draws in the guard band (and for rr_balance_keys).
//
// M = n / (n1 n0) ||G||^2 with G = sum_{i in T} X~_i (section 2.2; Appendix A remark), in
// FP64 on the whitened covariates.
#include <algorithm>

#include "rr_internal.h"

namespace rr {

// ---------------------------------------------------------------------------------------
// FP64 recomputation of M for listed draws: 16 draws per workgroup.  The four waves
// regenerate the treated sets into LDS; each thread then owns up to four covariates of a
// 1024-column group and adds the whitened rows of treated units in ascending unit order
// (row reads are coalesced and shared by the 16 draws); ||G||^2 is reduced per draw in a
// fixed order.
constexpr int kRecheckTile = 16;

// Workgroup wg of nwg takes the entry tiles wg, wg + nwg, ...
template <int S, bool EXACT>
__device__ __forceinline__ void recheck_run(const RecheckArgs& a, uint32_t wg, uint32_t nwg) {
    constexpr int WS = 8 * S + 1;
    __shared__ uint32_t bits[kRecheckTile][WS];
    __shared__ uint2 list[4][64];
    __shared__ double red[4][kRecheckTile];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const uint32_t cnt = *a.count;
    for (uint32_t e0 = wg * kRecheckTile; e0 < cnt; e0 += nwg * kRecheckTile) {
        const int nt = (int)min<uint32_t>(kRecheckTile, cnt - e0);
        for (int t = wave; t < kRecheckTile; t += 4) {
            if (t < nt) {
                if constexpr (EXACT) {
                    if (lane == 0) {
                        const uint64_t m = colex_unrank_mask(a.keys[e0 + t], a.n, a.n1, a.binom);
                        for (int w = 0; w < 8 * S; ++w) bits[t][w] = 0u;
                        bits[t][0] = (uint32_t)m;
                        bits[t][1] = (uint32_t)(m >> 32);
                    }
                } else {
                    gen_mc_bits<S>(a.seed, a.keys[e0 + t], a.n, a.n1, list[wave], bits[t]);
                }
            } else {
                for (int w = lane; w < 8 * S; w += 64) bits[t][w] = 0u;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        double part[kRecheckTile];
#pragma unroll
        for (int t = 0; t < kRecheckTile; ++t) part[t] = 0.0;
        for (int cg = 0; cg < a.d; cg += 1024) {
            double G[kRecheckTile][4];
#pragma unroll
            for (int t = 0; t < kRecheckTile; ++t)
#pragma unroll
                for (int c = 0; c < 4; ++c) G[t][c] = 0.0;
            for (int i = 0; i < a.n; ++i) {
                double x[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int col = cg + tid + 256 * c;
                    x[c] = col < a.d ? a.X64[(size_t)i * a.d + col] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < kRecheckTile; ++t) {
                    const uint32_t w = __builtin_amdgcn_readfirstlane(bits[t][i >> 5]);
                    if ((w >> (i & 31)) & 1u) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) G[t][c] += x[c];
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < kRecheckTile; ++t)
#pragma unroll
                for (int c = 0; c < 4; ++c) part[t] = fma(G[t][c], G[t][c], part[t]);
        }
#pragma unroll
        for (int t = 0; t < kRecheckTile; ++t) {
            const double v = wave_sum<double>(part[t]);
            if (lane == 0) red[wave][t] = v;
        }
        __syncthreads();
        if (tid < nt) a.out[e0 + tid] = a.scale * ((red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]));
        __syncthreads();
    }
}

template <int S, bool EXACT>
__global__ __launch_bounds__(256) void recheck_kernel(RecheckArgs a) {
    recheck_run<S, EXACT>(a, blockIdx.x, gridDim.x);
}

// Batched: pool tab[blockIdx.y], its entries strided over blockIdx.x.
template <int S>
__global__ __launch_bounds__(256) void recheck_batch_kernel(const RecheckArgs* tab) {
    recheck_run<S, false>(tab[blockIdx.y], blockIdx.x, gridDim.x);
}

hipError_t launch_recheck_batch(int S, const RecheckArgs* tab, int nprob, int gx, hipStream_t st) {
    const dim3 grid((unsigned)std::max(1, gx), (unsigned)nprob);
    switch (S) {
        case 1: hipLaunchKernelGGL((recheck_batch_kernel<1>), grid, dim3(256), 0, st, tab); break;
        case 2: hipLaunchKernelGGL((recheck_batch_kernel<2>), grid, dim3(256), 0, st, tab); break;
        case 4: hipLaunchKernelGGL((recheck_batch_kernel<4>), grid, dim3(256), 0, st, tab); break;
        case 8: hipLaunchKernelGGL((recheck_batch_kernel<8>), grid, dim3(256), 0, st, tab); break;
        case 16: hipLaunchKernelGGL((recheck_batch_kernel<16>), grid, dim3(256), 0, st, tab); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_recheck(int S, bool exact, const RecheckArgs& a, int grid, hipStream_t st) {
    grid = std::max(1, grid);
    if (exact) {
        hipLaunchKernelGGL((recheck_kernel<1, true>), dim3(grid), dim3(256), 0, st, a);
    } else {
        switch (S) {
            case 1: hipLaunchKernelGGL((recheck_kernel<1, false>), dim3(grid), dim3(256), 0, st, a); break;
            case 2: hipLaunchKernelGGL((recheck_kernel<2, false>), dim3(grid), dim3(256), 0, st, a); break;
            case 4: hipLaunchKernelGGL((recheck_kernel<4, false>), dim3(grid), dim3(256), 0, st, a); break;
            case 8: hipLaunchKernelGGL((recheck_kernel<8, false>), dim3(grid), dim3(256), 0, st, a); break;
            case 16: hipLaunchKernelGGL((recheck_kernel<16, false>), dim3(grid), dim3(256), 0, st, a); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace rr
