// Candidate generation: per-draw treated sets as bitmasks in HBM.
//
// Monte Carlo draws (section 2.3 generate_randomizations, "monte_carlo"; section 2.1
// "Key-only storage"): draw b treats the n1 units with the smallest Philox-4x32-10 unit
// keys (gen_mc_bits).  Exact enumeration (randomization_type = "exact"): draw r is the
// treated set of colex rank r.  One wave per Monte Carlo draw, one lane per exact draw.
#include <algorithm>

#include "rr_internal.h"

namespace rr {

// Register caps that keep three generation waves on every SIMD beside two contraction waves:
// up to 1024 units 64 registers (beside contraction waves of up to 168), up to 2048 units 96
// (beside the 1-block tiles of about 112; a few bytes spill).
template <int S, bool EXACT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S <= 4 ? 8 : (S == 8 ? 5 : 1)))) void gen_kernel(GenArgs g) {
    __shared__ uint2 slist[4][128];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    const uint64_t gw = (uint64_t)blockIdx.x * 4 + wave, nw = (uint64_t)gridDim.x * 4;
    if constexpr (EXACT) {
        for (uint64_t base = gw * 64; base < g.num; base += nw * 64) {
            const uint64_t idx = base + lane;
            if (idx < g.num) {
                const uint64_t key = g.keylist ? g.keylist[idx] : g.key_begin + idx;
                const uint64_t m = colex_unrank_mask(key, g.n, g.n1, g.binom);
                uint4* o = reinterpret_cast<uint4*>(g.out + idx * 8);
                o[0] = make_uint4((uint32_t)m, (uint32_t)(m >> 32), 0u, 0u);
                o[1] = make_uint4(0u, 0u, 0u, 0u);
            }
        }
    } else {
        for (uint64_t idx = gw; idx < g.num; idx += nw) {
            const uint64_t key = g.keylist ? g.keylist[idx] : g.key_begin + idx;
            gen_mc_bits_fixed<S>(g.seed, key, g.n, g.n1, slist[wave], g.out + idx * (8 * S));
            __builtin_amdgcn_wave_barrier();
        }
    }
}

hipError_t launch_gen(int S, bool exact, const GenArgs& g, int grid, hipStream_t st) {
    grid = std::max(1, grid);
    if (exact) {
        hipLaunchKernelGGL((gen_kernel<1, true>), dim3(grid), dim3(256), 0, st, g);
    } else {
        switch (S) {
            case 1: hipLaunchKernelGGL((gen_kernel<1, false>), dim3(grid), dim3(256), 0, st, g); break;
            case 2: hipLaunchKernelGGL((gen_kernel<2, false>), dim3(grid), dim3(256), 0, st, g); break;
            case 4: hipLaunchKernelGGL((gen_kernel<4, false>), dim3(grid), dim3(256), 0, st, g); break;
            case 8: hipLaunchKernelGGL((gen_kernel<8, false>), dim3(grid), dim3(256), 0, st, g); break;
            case 16: hipLaunchKernelGGL((gen_kernel<16, false>), dim3(grid), dim3(256), 0, st, g); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

// Batched generation over a table of pools: global draw index idx belongs to pool
// idx / per (draw idx % per of the pool's range).  One wave per draw.
template <int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(S <= 4 ? 8 : (S == 8 ? 5 : 1)))) void gen_batch_kernel(
    const GenArgs* tab, uint64_t total, uint64_t per) {
    __shared__ uint2 slist[4][128];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t gw = (uint64_t)blockIdx.x * 4 + wave, nw = (uint64_t)gridDim.x * 4;
    // (pool p, draw i) of idx, carried along the grid stride without a 64-bit division per draw
    uint64_t p = gw / per, i = gw - p * per;
    for (uint64_t idx = gw; idx < total; idx += nw) {
        const GenArgs& g = tab[p];
        gen_mc_bits_fixed<S, true>(g.seed, g.key_begin + i, g.n, g.n1, slist[wave], g.out + i * (8 * S));
        __builtin_amdgcn_wave_barrier();
        i += nw;
        while (i >= per) {
            i -= per;
            ++p;
        }
    }
}

hipError_t launch_gen_batch(int S, const GenArgs* tab, uint64_t nprob, uint64_t per, int grid, hipStream_t st) {
    grid = std::max(1, grid);
    const uint64_t total = nprob * per;
    switch (S) {
        case 1: hipLaunchKernelGGL((gen_batch_kernel<1>), dim3(grid), dim3(256), 0, st, tab, total, per); break;
        case 2: hipLaunchKernelGGL((gen_batch_kernel<2>), dim3(grid), dim3(256), 0, st, tab, total, per); break;
        case 4: hipLaunchKernelGGL((gen_batch_kernel<4>), dim3(grid), dim3(256), 0, st, tab, total, per); break;
        case 8: hipLaunchKernelGGL((gen_batch_kernel<8>), dim3(grid), dim3(256), 0, st, tab, total, per); break;
        case 16: hipLaunchKernelGGL((gen_batch_kernel<16>), dim3(grid), dim3(256), 0, st, tab, total, per); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Vector registers per lane of a Monte Carlo generation kernel (0 if unknown).
int gen_kernel_vgprs(int S, bool batch) {
    hipFuncAttributes fa{};
    hipError_t e = hipErrorInvalidValue;
    switch (S) {
#define RR_CASE(SV)                                                                              \
    case SV:                                                                                     \
        e = batch ? hipFuncGetAttributes(&fa, (const void*)gen_batch_kernel<SV>)                 \
                  : hipFuncGetAttributes(&fa, (const void*)gen_kernel<SV, false>);               \
        break;
        RR_CASE(1)
        RR_CASE(2)
        RR_CASE(4)
        RR_CASE(8)
        RR_CASE(16)
#undef RR_CASE
    }
    return e == hipSuccess ? fa.numRegs : 0;
}

int pow2_chunks(int n) {
    int c = (n + kUnitsPerChunk - 1) / kUnitsPerChunk;
    int S = 1;
    while (S < c) S <<= 1;
    return S;
}


// Regeneration of bitmasks (ceil(n/32) words per draw) from keys: one wave per draw.
template <int S, bool EXACT>
__global__ __launch_bounds__(256) void regen_kernel(const uint64_t* keys, uint64_t K, uint64_t seed,
                                                    int n, int n1, const uint64_t* binom,
                                                    uint32_t* out, int nw) {
    __shared__ uint32_t sbits[4][8 * kMaxS];
    __shared__ uint2 slist[4][128];
    const int wave = threadIdx.x >> 6, lane = lane_id();
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
        for (int w = lane; w < nw; w += 64) out[k * nw + w] = sbits[wave][w];
        __builtin_amdgcn_wave_barrier();
    }
}

hipError_t launch_regen(int S, bool exact, const uint64_t* keys, uint64_t K, uint64_t seed,
                        int n, int n1, const uint64_t* binom, uint32_t* out, int nw, int grid,
                        hipStream_t st) {
    if (exact) {
        hipLaunchKernelGGL((regen_kernel<1, true>), dim3(grid), dim3(256), 0, st, keys, K, seed, n, n1, binom, out, nw);
    } else {
        switch (S) {
            case 1: hipLaunchKernelGGL((regen_kernel<1, false>), dim3(grid), dim3(256), 0, st, keys, K, seed, n, n1, binom, out, nw); break;
            case 2: hipLaunchKernelGGL((regen_kernel<2, false>), dim3(grid), dim3(256), 0, st, keys, K, seed, n, n1, binom, out, nw); break;
            case 4: hipLaunchKernelGGL((regen_kernel<4, false>), dim3(grid), dim3(256), 0, st, keys, K, seed, n, n1, binom, out, nw); break;
            case 8: hipLaunchKernelGGL((regen_kernel<8, false>), dim3(grid), dim3(256), 0, st, keys, K, seed, n, n1, binom, out, nw); break;
            case 16: hipLaunchKernelGGL((regen_kernel<16, false>), dim3(grid), dim3(256), 0, st, keys, K, seed, n, n1, binom, out, nw); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace rr
