// FP64 recomputation of M for draws in the guard band (and for rr_balance_keys).
//
// M = n / (n1 n0) ||G||^2 with G = sum_{i in T} X~_i (section 2.2; Appendix A remark), in
// FP64 on the whitened covariates.  Exactly representable 0/1 weights make the FP64 matrix
// product W X~ the same sums, accumulated with FP64 roundings.
#include <algorithm>

#include "rr_internal.h"

namespace rr {

// ---------------------------------------------------------------------------------------
// FP64 recomputation of M for listed draws as the dense product G (draws x d) = W (draws x n,
// 0/1) X~ (n x d) on the FP64 matrix cores, in groups of 16 draws (v_mfma_f64_16x16x4f64:
// A lane l holds W[draw l % 16][unit 4k + l / 16], B lane l holds X~[unit 4k + l / 16][column
// l % 16], result item r of lane l is G[draw 4r + l / 16][column l % 16]).  A workgroup tile
// is 1 group, or 4 groups for long lists (the guard bands of problems with d >= n - 1): then
// each X~ fragment loaded feeds four MFMAs and X~ is read once per 64 draws, at the cost of
// more registers and fewer, longer tiles.  The four waves
// regenerate the treated sets into LDS, then split the 16-column blocks; each wave adds G^2
// of its blocks per draw and the partial sums are reduced in a fixed order (16 lanes, then
// the four waves), so the value depends neither on the launch shape nor on the tile size.

typedef double f64x4 __attribute__((ext_vector_type(4)));

struct RecheckShared {
    uint32_t* bits;        // [16 G][8 S + 1]
    uint2* list;           // [4][128]
    double* red;           // [4][16 G]
};

template <int S, bool EXACT, int G>
__device__ __forceinline__ void recheck_run(const RecheckArgs& a, uint32_t wg, uint32_t nwg, RecheckShared sh) {
    constexpr int WS = 8 * S + 1;
    constexpr int kRecheckGroups = G;
    constexpr int kRecheckTile = 16 * G;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    const uint32_t cnt = min(*a.count, a.cap);
    const int ncolb = (a.d + 15) / 16;
    const int nk = (a.n + 31) / 32;                 // 32-unit words of a bitmask
    constexpr uint32_t tile = kRecheckTile;
    for (uint32_t e0 = wg * tile; e0 < cnt; e0 += nwg * tile) {
        const int nt = (int)min<uint32_t>(tile, cnt - e0);
        for (int t = wave; t < (int)tile; t += 4) {
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
        // groups past the tile's draws skip their MFMAs (wave-uniform)
        const int ngroups = (nt + 15) / 16;
        double part[kRecheckGroups][4] = {};
        for (int cbk = wave; cbk < ncolb; cbk += 4) {
            const int col = 16 * cbk + c;
            const bool cval = col < a.d;
            const double* xcol = a.X64 + (cval ? col : 0);
            f64x4 acc[kRecheckGroups];
#pragma unroll
            for (int q = 0; q < kRecheckGroups; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
            for (int kw = 0; kw < nk; ++kw) {
                // 32 units = 8 K steps of 4; bitmask bits past n are zero
                uint32_t word[kRecheckGroups];
#pragma unroll
                for (int q = 0; q < kRecheckGroups; ++q) word[q] = sh.bits[(16 * q + c) * WS + kw];
#pragma unroll
                for (int st = 0; st < 8; ++st) {
                    const int unit = 32 * kw + 4 * st + g;
                    const double bv = (cval && unit < a.n) ? xcol[(size_t)unit * a.d] : 0.0;
#pragma unroll
                    for (int q = 0; q < kRecheckGroups; ++q) {
                        if (q < ngroups) {
                            const double av = ((word[q] >> (4 * st + g)) & 1u) ? 1.0 : 0.0;
                            acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
                        }
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < kRecheckGroups; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) part[q][r] = fma(acc[q][r], acc[q][r], part[q][r]);
        }
        // part[q][r] of lane (g, c): draw 16 q + 4 r + g, column c of this wave's blocks
#pragma unroll
        for (int q = 0; q < kRecheckGroups; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double v = part[q][r];
#pragma unroll
                for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
                if (c == 0) sh.red[wave * kRecheckTile + 16 * q + 4 * r + g] = v;
            }
        __syncthreads();
        if (tid < nt) {
            const double* rr = sh.red;
            a.out[e0 + tid] = a.scale * ((rr[tid] + rr[kRecheckTile + tid]) + (rr[2 * kRecheckTile + tid] + rr[3 * kRecheckTile + tid]));
        }
        __syncthreads();
    }
}

template <int S, bool EXACT, int G>
__device__ __forceinline__ void recheck_dispatch(const RecheckArgs& a, uint32_t wg, uint32_t nwg) {
    __shared__ uint32_t bits[16 * G * (8 * S + 1)];
    __shared__ uint2 list[4 * 128];
    __shared__ double red[4 * 16 * G];
    const RecheckShared sh{bits, list, red};
    recheck_run<S, EXACT, G>(a, wg, nwg, sh);
}

template <int S, bool EXACT>
__global__ __launch_bounds__(256) void recheck_kernel(RecheckArgs a) {
    recheck_dispatch<S, EXACT, 1>(a, blockIdx.x, gridDim.x);
}

// Batched: pool tab[blockIdx.y], its entries strided over blockIdx.x.
template <int S, int G>
__global__ __launch_bounds__(256) void recheck_batch_kernel(const RecheckArgs* tab) {
    recheck_dispatch<S, false, G>(tab[blockIdx.y], blockIdx.x, gridDim.x);
}

// Pools of up to 512 units (S <= 2) include every problem with d >= n - 1 in the batched
// workloads, whose bands are most of their draws: 64-draw tiles there, 16 elsewhere.
hipError_t launch_recheck_batch(int S, const RecheckArgs* tab, int nprob, int gx, hipStream_t st) {
    const dim3 grid((unsigned)std::max(1, gx), (unsigned)nprob);
    switch (S) {
        case 1: hipLaunchKernelGGL((recheck_batch_kernel<1, 4>), grid, dim3(256), 0, st, tab); break;
        case 2: hipLaunchKernelGGL((recheck_batch_kernel<2, 4>), grid, dim3(256), 0, st, tab); break;
        case 4: hipLaunchKernelGGL((recheck_batch_kernel<4, 1>), grid, dim3(256), 0, st, tab); break;
        case 8: hipLaunchKernelGGL((recheck_batch_kernel<8, 1>), grid, dim3(256), 0, st, tab); break;
        case 16: hipLaunchKernelGGL((recheck_batch_kernel<16, 1>), grid, dim3(256), 0, st, tab); break;
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
