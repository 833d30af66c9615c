// FP64 recomputation of M for draws in the guard band (and for rr_balance_keys).
//
// M = n / (n1 n0) ||G||^2 with G = sum_{i in T} X~_i (section 2.2; Appendix A remark), in
// FP64 on the whitened covariates; for the per-column criterion n / (n1 n0) max_j G_j^2.  Exactly representable 0/1 weights make the FP64 matrix
// product W X~ the same sums, accumulated with FP64 roundings.
#include <algorithm>

#include "rr_internal.h"

namespace rr {

// ---------------------------------------------------------------------------------------
// FP64 recomputation of M for listed draws as the dense product G (draws x d) = W (draws x n,
// 0/1) X~ (n x d) on the FP64 matrix cores, in groups of 16 draws (v_mfma_f64_16x16x4f64:
// A lane l holds W[draw l % 16][unit 4k + l / 16], B lane l holds X~[unit 4k + l / 16][column
// l % 16], result item r of lane l is G[draw 4r + l / 16][column l % 16]).  A workgroup tile
// is 1 group, or 4 groups in the batched launches for pools of up to 512 units, whose bands
// hold most draws of the problems with d >= n - 1: then each X~ fragment loaded feeds four
// MFMAs and X~ is read once per 64 draws, at the cost of more registers and fewer, longer
// tiles.  The NW = 4 waves of a workgroup regenerate the treated sets into LDS, then split
// the 16-column blocks, up to four at a time per wave (up to four independent MFMA chains,
// with the X~ loads of a whole bitmask word issued one word ahead); each wave adds G^2 of
// its blocks per draw and the partial sums are reduced in
// a fixed order (16 lanes, then the waves in index order), so the value depends neither on
// the launch shape nor on the tile size.
typedef double f64x4 __attribute__((ext_vector_type(4)));

struct RecheckShared {
    uint32_t* bits;        // [16 G][8 S + 1]
    uint2* list;           // [NW][128]
    double* red;           // [NW][16 G]
};

constexpr int recheck_waves(int) { return 4; }

// Column blocks cb0 + j NW, j < NB, of one wave: G^2 summed into part[q][r] (lane (g, c):
// draw 16 q + 4 r + g, column c of the block).
template <int NB, int G, int NW>
__device__ __forceinline__ void recheck_cols(const RecheckArgs& a, const uint32_t* bits, int WS, int cb0, int nk,
                                             int ngroups, int g, int c, double (&part)[G][4]) {
    typedef const __attribute__((address_space(1))) double* gptr;
    bool cval[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) cval[j] = 16 * (cb0 + j * NW) + c < a.d;
    f64x4 acc[NB][G];
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int q = 0; q < G; ++q) acc[j][q] = f64x4{0.0, 0.0, 0.0, 0.0};
    // The X~ values of one 32-unit bitmask word (8 K steps x NB blocks) are loaded as one
    // batch, unconditionally, and the next word's batch is issued before this word's MFMAs,
    // so a wave waits for memory about once per word rather than once per K step.  A K step
    // takes one row address; its blocks are fixed offsets from it.  Rows past n read row
    // n - 1 (their bits are zero, so they add nothing).  Lanes of columns past d read on past
    // the end of their row (at most 15 values; after the last row, into the zeroed padding
    // of X~): B column c only feeds result column c, which those lanes hold and leave out of
    // the sum of squares.
    const double* x0 = a.X64 + 16 * cb0 + c;
    const int nlast = a.n - 1;
    const size_t ld = (size_t)a.d;
    double buf0[8][NB], buf1[8][NB];
    auto load = [&](double (&b)[8][NB], int kw) {
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            const gptr p = (gptr)(x0 + (size_t)min(32 * kw + 4 * st + g, nlast) * ld);
#pragma unroll
            for (int j = 0; j < NB; ++j) b[st][j] = p[16 * NW * j];
        }
    };
    auto step = [&](const double (&b)[8][NB], int kw) {
        uint32_t word[G];
#pragma unroll
        for (int q = 0; q < G; ++q) word[q] = bits[(16 * q + c) * WS + kw];
#pragma unroll
        for (int st = 0; st < 8; ++st)
#pragma unroll
            for (int q = 0; q < G; ++q) {
                if (q < ngroups) {   // groups past the tile's draws (wave-uniform)
                    const double av = ((word[q] >> (4 * st + g)) & 1u) ? 1.0 : 0.0;
#pragma unroll
                    for (int j = 0; j < NB; ++j)
                        acc[j][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b[st][j], acc[j][q], 0, 0, 0);
                }
            }
    };
    load(buf0, 0);
    int kw = 0;
    for (; kw + 1 < nk; kw += 2) {
        load(buf1, kw + 1);
        step(buf0, kw);
        load(buf0, min(kw + 2, nk - 1));
        step(buf1, kw + 1);
    }
    if (kw < nk) step(buf0, kw);
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
        for (int q = 0; q < G; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (cval[j])
                    part[q][r] = a.maxmode ? fmax(part[q][r], acc[j][q][r] * acc[j][q][r])
                                           : fma(acc[j][q][r], acc[j][q][r], part[q][r]);
}

// Entries e0 .. min(e0 + 16 G, cnt) - 1 of the list (workgroup-uniform arguments).
template <int S, bool EXACT, int G>
__device__ __forceinline__ void recheck_tile(const RecheckArgs& a, uint32_t e0, uint32_t cnt, RecheckShared sh) {
    constexpr int NW = recheck_waves(S);
    constexpr int WS = 8 * S + 1;
    constexpr int kRecheckGroups = G;
    constexpr int kRecheckTile = 16 * G;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const int g = lane >> 4, c = lane & 15;
    const int ncolb = (a.d + 15) / 16;
    const int nk = (a.n + 31) / 32;                 // 32-unit words of a bitmask
    constexpr uint32_t tile = kRecheckTile;
    {
        const int nt = (int)min<uint32_t>(tile, cnt - e0);
        for (int t = wave; t < (int)tile; t += NW) {
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
        for (int e = tid; e < NW * kRecheckTile; e += blockDim.x) sh.red[e] = 0.0;
        __syncthreads();
        // groups past the tile's draws skip their MFMAs (wave-uniform)
        const int ngroups = (nt + 15) / 16;
        double part[kRecheckGroups][4] = {};
        // A wave takes its column blocks CBW at a time (blocks cb0 + j NW), so that each K
        // step issues up to CBW independent X~ loads and CBW x G independent MFMA chains; the
        // last group of a wave may hold fewer blocks (nb), and blocks past ncolb issue neither
        // loads nor MFMAs.
        constexpr int CBW = 4;
        for (int cb0 = wave; cb0 < ncolb; cb0 += NW * CBW) {
            const int nb = min(CBW, (ncolb - cb0 + NW - 1) / NW);   // wave-uniform, >= 1
            switch (nb) {
                case 1: recheck_cols<1, G, NW>(a, sh.bits, WS, cb0, nk, ngroups, g, c, part); break;
                case 2: recheck_cols<2, G, NW>(a, sh.bits, WS, cb0, nk, ngroups, g, c, part); break;
                case 3: recheck_cols<3, G, NW>(a, sh.bits, WS, cb0, nk, ngroups, g, c, part); break;
                default: recheck_cols<4, G, NW>(a, sh.bits, WS, cb0, nk, ngroups, g, c, part); break;
            }
        }
        // part[q][r] of lane (g, c): draw 16 q + 4 r + g, column c of this wave's blocks
#pragma unroll
        for (int q = 0; q < kRecheckGroups; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double v = part[q][r];
#pragma unroll
                for (int o = 8; o >= 1; o >>= 1) {
                    const double u = __shfl_xor(v, o, 64);
                    v = a.maxmode ? fmax(v, u) : v + u;
                }
                if (c == 0) sh.red[wave * kRecheckTile + 16 * q + 4 * r + g] = v;
            }
        __syncthreads();
        if (tid < nt) {
            double v = sh.red[tid];
#pragma unroll
            for (int w = 1; w < NW; ++w) v = a.maxmode ? fmax(v, sh.red[w * kRecheckTile + tid]) : v + sh.red[w * kRecheckTile + tid];
            a.out[e0 + tid] = a.scale * v;
        }
        __syncthreads();
    }
}

#define RR_RECHECK_SHARED(S, G)                                  \
    __shared__ uint32_t bits[16 * (G) * (8 * (S) + 1)];           \
    __shared__ uint2 list[recheck_waves(S) * 128];               \
    __shared__ double red[recheck_waves(S) * 16 * (G)];          \
    const RecheckShared sh{bits, list, red};

template <int S, bool EXACT>
__global__ __launch_bounds__(64 * recheck_waves(S)) void recheck_kernel(RecheckArgs a) {
    RR_RECHECK_SHARED(S, 1)
    const uint32_t cnt = min(*a.count, a.cap);
    for (uint32_t e0 = blockIdx.x * 16u; e0 < cnt; e0 += gridDim.x * 16u) recheck_tile<S, EXACT, 1>(a, e0, cnt, sh);
}

// Batched: one flat list of the tiles of all pools of a bitmask class.  offs[p] is the
// first tile of pool p (offs[nprob] the total), written by recheck_offsets_kernel from the
// pools' list lengths; workgroups stride over the tiles, so every pool's band is spread over
// the whole GPU whatever its length.
template <int S, int G>
__global__ __launch_bounds__(64 * recheck_waves(S)) void recheck_batch_kernel(const RecheckArgs* tab, int nprob,
                                                                             const uint32_t* offs) {
    RR_RECHECK_SHARED(S, G)
    const uint32_t total = offs[nprob];
    for (uint32_t T = blockIdx.x; T < total; T += gridDim.x) {
        int lo = 0, hi = nprob;   // offs[lo] <= T < offs[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (offs[mid] <= T) lo = mid; else hi = mid;
        }
        const RecheckArgs& a = tab[lo];
        const uint32_t cnt = min(*a.count, a.cap);
        recheck_tile<S, false, G>(a, (T - offs[lo]) * (16u * G), cnt, sh);
    }
}
#undef RR_RECHECK_SHARED

// offs[p + 1] = offs[p] + ceil(len_p / tile), offs[0] = 0.  One wave (it must not wait for a
// large slot while the other stream's rechecks hold the CUs), 64 pools per step.
__global__ __launch_bounds__(64) void recheck_offsets_kernel(const RecheckArgs* tab, int nprob, uint32_t tile,
                                                             uint32_t* offs) {
    const int lane = threadIdx.x;
    uint32_t base = 0;
    for (int c0 = 0; c0 < nprob; c0 += 64) {
        const int i = c0 + lane;
        uint32_t v = i < nprob ? (min(*tab[i].count, tab[i].cap) + tile - 1) / tile : 0u;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(v, o, 64);
            if (lane >= o) v += t;
        }
        if (i < nprob) offs[i + 1] = base + v;
        base += __shfl(v, 63, 64);
    }
    if (lane == 0) offs[0] = 0;
}

// Pools of up to 512 units (S <= 2) include every problem with d >= n - 1 in the batched
// workloads, whose bands are most of their draws: 64-draw tiles there, 16 elsewhere.
hipError_t launch_recheck_batch(int S, const RecheckArgs* tab, int nprob, uint32_t* offs, int grid, hipStream_t st) {
    grid = std::max(1, grid);
    const uint32_t tile = S <= 2 ? 64u : 16u;
    hipLaunchKernelGGL(recheck_offsets_kernel, dim3(1), dim3(64), 0, st, tab, nprob, tile, offs);
    switch (S) {
        case 1: hipLaunchKernelGGL((recheck_batch_kernel<1, 4>), dim3(grid), dim3(64 * recheck_waves(1)), 0, st, tab, nprob, offs); break;
        case 2: hipLaunchKernelGGL((recheck_batch_kernel<2, 4>), dim3(grid), dim3(64 * recheck_waves(2)), 0, st, tab, nprob, offs); break;
        case 4: hipLaunchKernelGGL((recheck_batch_kernel<4, 1>), dim3(grid), dim3(64 * recheck_waves(4)), 0, st, tab, nprob, offs); break;
        case 8: hipLaunchKernelGGL((recheck_batch_kernel<8, 1>), dim3(grid), dim3(64 * recheck_waves(8)), 0, st, tab, nprob, offs); break;
        case 16: hipLaunchKernelGGL((recheck_batch_kernel<16, 1>), dim3(grid), dim3(64 * recheck_waves(16)), 0, st, tab, nprob, offs); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_recheck(int S, bool exact, const RecheckArgs& a, int grid, hipStream_t st) {
    grid = std::max(1, grid);
    if (exact) {
        hipLaunchKernelGGL((recheck_kernel<1, true>), dim3(grid), dim3(64 * recheck_waves(1)), 0, st, a);
    } else {
        switch (S) {
            case 1: hipLaunchKernelGGL((recheck_kernel<1, false>), dim3(grid), dim3(64 * recheck_waves(1)), 0, st, a); break;
            case 2: hipLaunchKernelGGL((recheck_kernel<2, false>), dim3(grid), dim3(64 * recheck_waves(2)), 0, st, a); break;
            case 4: hipLaunchKernelGGL((recheck_kernel<4, false>), dim3(grid), dim3(64 * recheck_waves(4)), 0, st, a); break;
            case 8: hipLaunchKernelGGL((recheck_kernel<8, false>), dim3(grid), dim3(64 * recheck_waves(8)), 0, st, a); break;
            case 16: hipLaunchKernelGGL((recheck_kernel<16, false>), dim3(grid), dim3(64 * recheck_waves(16)), 0, st, a); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace rr
