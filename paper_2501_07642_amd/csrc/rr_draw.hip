// Fused candidate generation + balance contraction + acceptance prefilter, and the FP64
// recomputation of M for draws near the acceptance boundary.
//
// Method (section 2.2, Appendix A remark): with X~ = (X - 1 mu^T) L^-T the centred,
// whitened covariates, the treated sum G = sum_{i in T} X~_i = W X~ (W the 0/1 row of the
// draw) gives M = n / (n1 n0) * ||G||^2 (chi^2_d scale).  Centring makes the control sum
// redundant: sum_{i in C} X~_i = -G.
//
// Per wave: a tile of 32 * DB draws.  Generation fills the tile's bitmasks in LDS (one draw
// at a time, 64 lanes per draw).  Contraction computes G^T = X~^T W^T on MFMA: the A
// operand is a 32-covariate x 16-unit block of X~^T read from the precomputed operand
// records, the B operand is the 16-unit x 32-draw block of W^T expanded from bits.  In
// the output block, lane l holds draw l % 32 and 16 covariates, so ||G||^2 is reduced in
// registers and across the two lane halves.
#include "rr_internal.h"

namespace rr {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;

enum { GEN_MC_RANGE = 0, GEN_MC_LIST = 1, GEN_EXACT_RANGE = 2, GEN_EXACT_LIST = 3 };


__device__ __forceinline__ uint4 expand_bf16(uint32_t x) {
    // 8 bits -> 8 BF16 values (1.0 = 0x3F80 or 0): bit 2k -> low half of dword k,
    // bit 2k+1 -> high half.  y holds bit i at i and at i + 15.
    const uint32_t y = x | (x << 15);
    uint4 r;
    r.x = __umul24(y & 0x00010001u, 0x3F80u);
    r.y = __umul24(y & 0x00040004u, 0x3F80u >> 2);
    r.z = __umul24(y & 0x00100010u, 0x3F80u >> 4);
    r.w = __umul24(y & 0x00400040u, 0x3F80u >> 6);
    return r;
}

template <int S>
__device__ __forceinline__ void gen_tile_mc(const DrawArgs& a, uint64_t tile0, int count,
                                            uint32_t* bits, int wstr, uint32_t* hist,
                                            uint2* list, bool from_list) {
    const int lane = lane_id();
    for (int dl = 0; dl < count; ++dl) {
        const uint64_t idx = tile0 + dl;
        uint32_t* out = bits + dl * wstr;
        if (idx < a.num) {
            const uint64_t key = from_list ? a.keylist[idx] : a.key_begin + idx;
            gen_mc_bits<S>(a.seed, key, a.n, a.n1, hist, list, out);
        } else {
            for (int w = lane; w < 8 * S; w += 64) out[w] = 0u;
        }
    }
}

__device__ __forceinline__ void gen_tile_exact(const DrawArgs& a, uint64_t tile0, int count,
                                               uint32_t* bits, int wstr, bool from_list) {
    const int lane = lane_id();
    for (int base = 0; base < count; base += 64) {
        const int dl = base + lane;
        if (dl < count) {
            const uint64_t idx = tile0 + dl;
            uint64_t m = 0;
            if (idx < a.num) {
                const uint64_t key = from_list ? a.keylist[idx] : a.key_begin + idx;
                m = colex_unrank_mask(key, a.n, a.n1, a.binom);
            }
            uint32_t* out = bits + dl * wstr;
            out[0] = (uint32_t)m;
            out[1] = (uint32_t)(m >> 32);
            for (int w = 2; w < 8; ++w) out[w] = 0u;
        }
    }
}

template <int S, int PREC, int GEN, int CB, int DB>
__global__ __launch_bounds__(256) void draw_kernel(DrawArgs a) {
    constexpr int TILE = 32 * DB;
    constexpr int WSTR = 8 * S + 1;          // +1 word: draws of a block hit distinct banks
    extern __shared__ uint32_t smem[];
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5;                 // lane half: K sub-block in operands
    const int j = lane & 31;                 // draw column within a 32-draw block
    uint32_t* bits = smem + wave * (TILE * WSTR + 256 + 128);
    uint32_t* hist = bits + TILE * WSTR;
    uint2* list = reinterpret_cast<uint2*>(hist + 256);

    const uint64_t ntiles = (a.num + TILE - 1) / TILE;
    const uint64_t nwaves = (uint64_t)gridDim.x * 4;
    for (uint64_t t = (uint64_t)blockIdx.x * 4 + wave; t < ntiles; t += nwaves) {
        const uint64_t tile0 = t * TILE;
        if constexpr (GEN == GEN_EXACT_RANGE || GEN == GEN_EXACT_LIST)
            gen_tile_exact(a, tile0, TILE, bits, WSTR, GEN == GEN_EXACT_LIST);
        else
            gen_tile_mc<S>(a, tile0, TILE, bits, WSTR, hist, list, GEN == GEN_MC_LIST);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();

        float ss[DB], sa[DB];
#pragma unroll
        for (int db = 0; db < DB; ++db) ss[db] = sa[db] = 0.f;

        for (int c0 = 0; c0 < a.ncb; c0 += CB) {
            f32x16 acc[CB][DB];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int db = 0; db < DB; ++db)
#pragma unroll
                    for (int e = 0; e < 16; ++e) acc[cb][db][e] = 0.f;

            for (int k = 0; k < a.ks; ++k) {
                const uint4* rec = a.op + ((size_t)k * a.ncb + c0) * kRecordU4;
                uint32_t byte2[DB];
#pragma unroll
                for (int db = 0; db < DB; ++db) {
                    const uint32_t w = bits[(32 * db + j) * WSTR + (k >> 1)];
                    byte2[db] = (w >> (16 * (k & 1))) & 0xFFFFu;   // units 16k .. 16k+15
                }
                if constexpr (PREC == RR_PREC_SPLIT_BF16) {
                    bf16x8 bw[DB];
#pragma unroll
                    for (int db = 0; db < DB; ++db) {
                        const uint4 e = expand_bf16((byte2[db] >> (8 * h)) & 0xFFu);
                        bw[db] = __builtin_bit_cast(bf16x8, e);
                    }
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        const bf16x8 ahi = __builtin_bit_cast(bf16x8, rec[cb * kRecordU4 + lane]);
                        const bf16x8 alo = __builtin_bit_cast(bf16x8, rec[cb * kRecordU4 + 64 + lane]);
#pragma unroll
                        for (int db = 0; db < DB; ++db) {
                            acc[cb][db] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ahi, bw[db], acc[cb][db], 0, 0, 0);
                            acc[cb][db] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(alo, bw[db], acc[cb][db], 0, 0, 0);
                        }
                    }
                } else {
                    // FP32 form: each K step starts from a zero accumulator and is added to
                    // the running total on the VALU, so the rounding chain of an output is
                    // 16 steps inside the K step plus one add per K step.
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        f32x16 st[DB];
#pragma unroll
                        for (int db = 0; db < DB; ++db)
#pragma unroll
                            for (int e = 0; e < 16; ++e) st[db][e] = 0.f;
#pragma unroll
                        for (int p = 0; p < 2; ++p) {
                            const uint4 av = rec[cb * kRecordU4 + 64 * p + lane];
                            const float af[4] = {__uint_as_float(av.x), __uint_as_float(av.y),
                                                 __uint_as_float(av.z), __uint_as_float(av.w)};
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
#pragma unroll
                                for (int db = 0; db < DB; ++db) {
                                    const float bv = (float)((byte2[db] >> (8 * p + 2 * q + h)) & 1u);
                                    st[db] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[q], bv, st[db], 0, 0, 0);
                                }
                            }
                        }
#pragma unroll
                        for (int db = 0; db < DB; ++db) acc[cb][db] += st[db];
                    }
                }
            }
            // ||G||^2 and sum |G_j| cabs_j over this chunk's covariates.
#pragma unroll
            for (int db = 0; db < DB; ++db) {
                float s2 = 0.f, s1 = 0.f;
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const int cov0 = 32 * (c0 + cb) + 4 * h;
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const float g = acc[cb][db][r];
                        const int cov = cov0 + 8 * (r >> 2) + (r & 3);
                        s2 = fmaf(g, g, s2);
                        s1 = fmaf(fabsf(g), a.cabs[cov], s1);
                    }
                }
                ss[db] += s2;
                sa[db] += s1;
            }
        }

#pragma unroll
        for (int db = 0; db < DB; ++db) {
            const float s2 = ss[db] + __shfl_xor(ss[db], 32, 64);
            const float s1 = sa[db] + __shfl_xor(sa[db], 32, 64);
            const uint64_t idx = tile0 + 32 * db + j;
            const bool live = h == 0 && idx < a.num;
            const float m32 = a.scale * s2;
            const float err = a.safety * (a.scale * (a.two_kappa * s1 + a.csq) + a.gamma_ss * m32);
            if (a.out_m32) {
                if (live) {
                    a.out_m32[idx] = m32;
                    a.out_err[idx] = err;
                }
            } else {
                const float hi = (m32 + err) * (1.0f + 0x1p-21f);
                const float lo = fmaxf((m32 - err) * (1.0f - 0x1p-21f), 0.0f);
                const bool pass = live && (a.U == nullptr || lo <= *a.U);
                const uint64_t bm = ballot(pass);
                if (bm) {
                    uint32_t base = 0;
                    if (lane == (int)__builtin_ctzll(bm))
                        base = atomicAdd(a.cand_count, (uint32_t)__builtin_popcountll(bm));
                    base = __shfl(base, (int)__builtin_ctzll(bm), 64);
                    if (pass) {
                        const uint32_t pos = base + __builtin_amdgcn_mbcnt_hi(
                                                        (uint32_t)(bm >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
                        if (pos < a.cand_cap) {
                            a.cand_key[pos] = GEN == GEN_MC_LIST || GEN == GEN_EXACT_LIST
                                                  ? a.keylist[idx]
                                                  : a.key_begin + idx;
                            a.cand_hi[pos] = hi;
                            a.cand_lo[pos] = lo;
                            a.cand_m[pos] = m32;
                        }
                    }
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------------------------------
// FP64 recomputation of M for listed draws: 16 draws per workgroup.  The four waves
// regenerate the treated sets into LDS; each thread then owns up to four covariates of a
// 1024-column group and adds the whitened rows of treated units in ascending unit order
// (row reads are coalesced and shared by the 16 draws); ||G||^2 is reduced per draw in a
// fixed order.
constexpr int kRecheckTile = 16;

template <int S, bool EXACT>
__global__ __launch_bounds__(256) void recheck_kernel(RecheckArgs a) {
    constexpr int WS = 8 * S + 1;
    __shared__ uint32_t bits[kRecheckTile][WS];
    __shared__ uint32_t hist[4][256];
    __shared__ uint2 list[4][64];
    __shared__ double red[4][kRecheckTile];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const uint32_t cnt = *a.count;
    for (uint32_t e0 = blockIdx.x * kRecheckTile; e0 < cnt; e0 += gridDim.x * kRecheckTile) {
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
                    gen_mc_bits<S>(a.seed, a.keys[e0 + t], a.n, a.n1, hist[wave], list[wave], bits[t]);
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

// ---------------------------------------------------------------------------------------
// Host-side launchers.
constexpr int kDB = 2;
// covariate blocks per chunk: the FP32 form keeps a second accumulator set per K step
constexpr int cb_for(int prec) { return prec == RR_PREC_SPLIT_BF16 ? 4 : 2; }

size_t draw_lds_bytes(int S) { return 4 * ((32 * kDB) * (8 * S + 1) + 256 + 128) * sizeof(uint32_t); }

template <int S, int PREC, int GEN>
static hipError_t launch_draw_t(const DrawArgs& a, int grid, hipStream_t st) {
    auto k = draw_kernel<S, PREC, GEN, cb_for(PREC), kDB>;
    const size_t lds = draw_lds_bytes(S);
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(grid), dim3(256), lds, st, a);
    return hipGetLastError();
}

template <int PREC, int GEN>
static hipError_t launch_draw_s(int S, const DrawArgs& a, int grid, hipStream_t st) {
    switch (S) {
        case 1: return launch_draw_t<1, PREC, GEN>(a, grid, st);
        case 2: return launch_draw_t<2, PREC, GEN>(a, grid, st);
        case 4: return launch_draw_t<4, PREC, GEN>(a, grid, st);
        case 8: return launch_draw_t<8, PREC, GEN>(a, grid, st);
        case 16: return launch_draw_t<16, PREC, GEN>(a, grid, st);
    }
    return hipErrorInvalidValue;
}

int pow2_chunks(int n) {
    int c = (n + kUnitsPerChunk - 1) / kUnitsPerChunk;
    int S = 1;
    while (S < c) S <<= 1;
    return S;
}

hipError_t launch_draw(int S, int prec, bool exact, bool from_list, const DrawArgs& a,
                       int grid, hipStream_t st) {
    if (exact) {
        if (prec == RR_PREC_SPLIT_BF16)
            return from_list ? launch_draw_t<1, RR_PREC_SPLIT_BF16, GEN_EXACT_LIST>(a, grid, st)
                             : launch_draw_t<1, RR_PREC_SPLIT_BF16, GEN_EXACT_RANGE>(a, grid, st);
        return from_list ? launch_draw_t<1, RR_PREC_FP32, GEN_EXACT_LIST>(a, grid, st)
                         : launch_draw_t<1, RR_PREC_FP32, GEN_EXACT_RANGE>(a, grid, st);
    }
    if (prec == RR_PREC_SPLIT_BF16)
        return from_list ? launch_draw_s<RR_PREC_SPLIT_BF16, GEN_MC_LIST>(S, a, grid, st)
                         : launch_draw_s<RR_PREC_SPLIT_BF16, GEN_MC_RANGE>(S, a, grid, st);
    return from_list ? launch_draw_s<RR_PREC_FP32, GEN_MC_LIST>(S, a, grid, st)
                     : launch_draw_s<RR_PREC_FP32, GEN_MC_RANGE>(S, a, grid, st);
}

int draw_tile() { return 32 * kDB; }
int draw_cb(int prec) { return cb_for(prec); }

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

// Regeneration of bitmasks (ceil(n/32) words per draw) from keys: one wave per draw.
template <int S, bool EXACT>
__global__ __launch_bounds__(256) void regen_kernel(const uint64_t* keys, uint64_t K, uint64_t seed,
                                                    int n, int n1, const uint64_t* binom,
                                                    uint32_t* out, int nw) {
    __shared__ uint32_t sbits[4][8 * kMaxS];
    __shared__ uint32_t shist[4][256];
    __shared__ uint2 slist[4][64];
    const int wave = threadIdx.x >> 6, lane = lane_id();
    for (uint64_t k = (uint64_t)blockIdx.x * 4 + wave; k < K; k += (uint64_t)gridDim.x * 4) {
        if constexpr (EXACT) {
            if (lane == 0) {
                const uint64_t m = colex_unrank_mask(keys[k], n, n1, binom);
                sbits[wave][0] = (uint32_t)m;
                sbits[wave][1] = (uint32_t)(m >> 32);
            }
        } else {
            gen_mc_bits<S>(seed, keys[k], n, n1, shist[wave], slist[wave], sbits[wave]);
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
