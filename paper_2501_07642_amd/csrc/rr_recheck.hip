// FP64 recomputation of M for draws in the guard band (and for rr_balance_keys).
//
// M = n / (n1 n0) ||G||^2 with G = sum_{i in T} X~_i (section 2.2; Appendix A remark), in
// FP64 on the whitened covariates.
#include <algorithm>

#include "rr_internal.h"

namespace rr {

// ---------------------------------------------------------------------------------------
// FP64 recomputation of M for listed draws: 16 draws per workgroup tile.  The four waves
// regenerate the treated sets into LDS; the threads then add the whitened rows of treated
// units in ascending unit order, covariates split over the threads in column groups of CW
// (row reads are coalesced and shared by the draws), and ||G||^2 is reduced per draw in a
// fixed order.  The column-group width follows d so that few lanes idle:
//   CW = 1024: every thread owns 4 columns and all 16 draws;
//   CW = 256:  every thread owns 1 column and all 16 draws;
//   CW = 64:   wave q owns draws 4q .. 4q+3, every lane 1 column.
constexpr int kRecheckTile = 16;

struct RecheckShared {
    uint32_t* bits;        // [kRecheckTile][8 S + 1]
    uint2* list;           // [4][128]
    double* red;           // [4][kRecheckTile]
};

template <int S, bool EXACT, int CW>
__device__ __forceinline__ void recheck_run(const RecheckArgs& a, uint32_t wg, uint32_t nwg, RecheckShared sh) {
    constexpr int WS = 8 * S + 1;
    constexpr int TW = CW < 256 ? CW : 256;                 // threads across one column group row
    constexpr int CPT = CW / TW;                            // columns per thread
    constexpr int DT = CW < 256 ? kRecheckTile / 4 : kRecheckTile;   // draws per thread
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const int d0 = CW < 256 ? DT * wave : 0;                // first draw of this thread
    const int c0 = tid % TW;
    const uint32_t cnt = *a.count;
    for (uint32_t e0 = wg * kRecheckTile; e0 < cnt; e0 += nwg * kRecheckTile) {
        const int nt = (int)min<uint32_t>(kRecheckTile, cnt - e0);
        for (int t = wave; t < kRecheckTile; t += 4) {
            uint32_t* bt = sh.bits + t * WS;
            if (t < nt) {
                if constexpr (EXACT) {
                    if (lane == 0) {
                        const uint64_t m = colex_unrank_mask(a.keys[e0 + t], a.n, a.n1, a.binom);
                        for (int w = 0; w < 8 * S; ++w) bt[w] = 0u;
                        bt[0] = (uint32_t)m;
                        bt[1] = (uint32_t)(m >> 32);
                    }
                } else {
                    gen_mc_bits_fixed<S>(a.seed, a.keys[e0 + t], a.n, a.n1, sh.list + 128 * wave, bt);
                }
            } else {
                for (int w = lane; w < 8 * S; w += 64) bt[w] = 0u;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        for (int e = tid; e < 4 * kRecheckTile; e += blockDim.x) sh.red[e] = 0.0;
        __syncthreads();
        double part[DT];
#pragma unroll
        for (int t = 0; t < DT; ++t) part[t] = 0.0;
        for (int cg = 0; cg < a.d; cg += CW) {
            double G[DT][CPT];
#pragma unroll
            for (int t = 0; t < DT; ++t)
#pragma unroll
                for (int c = 0; c < CPT; ++c) G[t][c] = 0.0;
            for (int i = 0; i < a.n; ++i) {
                double x[CPT];
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const int col = cg + c0 + TW * c;
                    x[c] = col < a.d ? a.X64[(size_t)i * a.d + col] : 0.0;
                }
#pragma unroll
                for (int t = 0; t < DT; ++t) {
                    const uint32_t w = __builtin_amdgcn_readfirstlane(sh.bits[(d0 + t) * WS + (i >> 5)]);
                    if ((w >> (i & 31)) & 1u) {
#pragma unroll
                        for (int c = 0; c < CPT; ++c) G[t][c] += x[c];
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < DT; ++t)
#pragma unroll
                for (int c = 0; c < CPT; ++c) part[t] = fma(G[t][c], G[t][c], part[t]);
        }
#pragma unroll
        for (int t = 0; t < DT; ++t) {
            const double v = wave_sum<double>(part[t]);
            if (lane == 0) sh.red[wave * kRecheckTile + d0 + t] = v;
        }
        __syncthreads();
        if (tid < nt) {
            const double* r = sh.red;
            a.out[e0 + tid] = a.scale * ((r[tid] + r[kRecheckTile + tid]) + (r[2 * kRecheckTile + tid] + r[3 * kRecheckTile + tid]));
        }
        __syncthreads();
    }
}

template <int S, bool EXACT>
__device__ __forceinline__ void recheck_dispatch(const RecheckArgs& a, uint32_t wg, uint32_t nwg) {
    __shared__ uint32_t bits[kRecheckTile * (8 * S + 1)];
    __shared__ uint2 list[4 * 128];
    __shared__ double red[4 * kRecheckTile];
    const RecheckShared sh{bits, list, red};
    if (a.d <= 64)
        recheck_run<S, EXACT, 64>(a, wg, nwg, sh);
    else if (a.d <= 256)
        recheck_run<S, EXACT, 256>(a, wg, nwg, sh);
    else
        recheck_run<S, EXACT, 1024>(a, wg, nwg, sh);
}

template <int S, bool EXACT>
__global__ __launch_bounds__(256) void recheck_kernel(RecheckArgs a) {
    recheck_dispatch<S, EXACT>(a, blockIdx.x, gridDim.x);
}

// Batched: pool tab[blockIdx.y], its entries strided over blockIdx.x.
template <int S>
__global__ __launch_bounds__(256) void recheck_batch_kernel(const RecheckArgs* tab) {
    recheck_dispatch<S, false>(tab[blockIdx.y], blockIdx.x, gridDim.x);
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
