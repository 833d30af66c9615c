// Balance contraction: M for every candidate draw from its bitmask, on MFMA.
//
// Method (section 2.2, Appendix A remark): with X~ = (X - 1 mu^T) L^-T the centred,
// whitened covariates, the treated sum G = sum_{i in T} X~_i = W X~ (W the 0/1 row of the
// draw) gives M = n / (n1 n0) ||G||^2 (chi^2_d scale).  Centring makes the control sum
// redundant: sum_{i in C} X~_i = -G.
//
// One workgroup (NW waves) takes a tile of 32 NW DB draws; wave w owns draws
// [32 DB w, 32 DB (w+1)).  G^T = X~^T W^T is computed per covariate chunk of 32 CB: the A
// operand (32 covariates x 16 units of X~^T) comes from the precomputed operand records,
// staged from global memory straight into LDS eight K steps at a time (double-buffered,
// shared by the waves of the workgroup; the barrier that hands a stage over sits before its
// last K step in the MFMA-16 forms); the B operand (16 units x 32 draws of W^T) is expanded
// from the tile's bitmasks in LDS.  In the split and Gram forms a K step's MFMAs run on
// registers filled during the step before: its A fragments are read from LDS and its B
// fragments expanded there, half an expansion after each MFMA; the split form also reads a
// stage's bitmask words during the stage before and expands its first B fragments in that
// stage's last step, so every stage starts on MFMAs.
// In an output block, lane l holds draw l % 32 and 16 covariates, so ||G||^2 is reduced in
// registers and across the two lane halves; the error bounds need only ||G|| (or, for the
// Gram form, the sum of |G'_j| over the treated units).  For the per-column criterion
// (maxmode) the same reduction takes the largest G_j^2 instead of the sum.
//
//   split BF16: X~ = hi + lo, two 32x32x16 BF16 MFMA per K step into one FP32 accumulator;
//   FP32:       32x32x2 FP32 MFMA; each K step starts from zero and is added on the VALU;
//   Gram:       the split form with K = X~ X~^T (n x n) in place of X~: G'_j = sum_{i in T} K_ij
//               for every unit j, and M = n / (n1 n0) sum_{j in T} G'_j (the epilogue reads
//               the treated bits of its rows from the tile's bitmasks); n^2 instead of n d work;
//   fixed I8:   X~ = s (128 hi + lo) per block of 32 covariates; the A operand holds the
//               digits (-hi, lo) of 16 units, the B operand the bytes (-128, 1) of each
//               treated unit, so one 32x32x32 int8 MFMA per K step sums 128 hi + lo exactly
//               in int32; the chunk epilogue scales by s in FP32.
#include <algorithm>
#include <type_traits>

#include "rr_internal.h"

namespace rr {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;

constexpr int kKStage = kKStepsPerStage;   // K steps per LDS stage

// Split form: W enters as 2.0 (BF16 0x4000, a single bit per half) so that a B dword is a
// rotation and a mask of the bitmask word: the operand records pair units u and u + 16 in a
// dword (both bits 16 apart), and with xr = the word rotated right by 4h, dword t of K step
// parity p is rotr(xr, 8p + t + 18) & 0x40004000 (unit bits land on 14 and 30).  G comes
// out as 2G exactly, and the sum of squares is scaled back by 1/4 (exact).
template <int P, int T>
__device__ __forceinline__ uint32_t wdword_split(uint32_t xr) {
    return __builtin_amdgcn_alignbit(xr, xr, (8 * P + T + 18) & 31) & 0x40004000u;
}

// 8 bits -> 8 unit byte pairs (-128, 1) = 0x0180 per treated unit, 0 otherwise: bit 2t ->
// low half of dword t, bit 2t + 1 -> high half.  y holds bit i at i and at i + 15.
__device__ __forceinline__ uint4 expand_i8(uint32_t x) {
    const uint32_t y = x | (x << 15);
    uint4 r;
    r.x = __umul24(y & 0x00010001u, 0x0180u);
    r.y = __umul24(y & 0x00040004u, 0x0180u >> 2);
    r.z = __umul24(y & 0x00100010u, 0x0180u >> 4);
    r.w = __umul24(y & 0x00400040u, 0x0180u >> 6);
    return r;
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// word 3 of a raw buffer resource on gfx9-family parts: 32-bit data format, no swizzle
constexpr int kBufferWord3 = 0x00020000;

constexpr int planes_for(int prec) { return prec == RR_PREC_FIXED_I8 ? 1 : 2; }

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }
// A pointer every lane of the wave holds (a batched tile's operand records come from a table
// in memory, so the compiler cannot see that): in scalar registers, as a buffer resource needs.
template <typename T>
__device__ __forceinline__ const T* uniform_ptr(const T* p) {
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const T*)(uintptr_t)(((uint64_t)hi << 32) | lo);
}

template <int PREC, int NW, int CB, int DB, int S, bool BATCH>
// 8-wave tiles: at most 168 registers per wave (two waves per SIMD, 336 of the 512 registers),
// which leaves three 64-register generation waves per SIMD beside them.
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(NW == 8 ? 3 : NW / 2)))
void contract_kernel(ContractArgs a0) {
    constexpr int TILE = NW * 32 * DB;
    // Stage barrier of the one-plane and two-plane MFMA forms: it sits before the last K step of
    // a stage, whose operands are then already in registers, so that the waves of a SIMD, which
    // leave every barrier together, restart on those MFMAs rather than on LDS reads; the copy of
    // stage gs + 2 into the buffer stage gs has left follows them.  (The FP32 form keeps the
    // barrier at the end of the stage.)
    constexpr bool kEarly = PREC != RR_PREC_FP32;
    constexpr int WSTR = 8 * S + 1;                       // +1: 32 draws hit 32 banks
    constexpr bool kGram = PREC == RR_PREC_GRAM_BF16;
    constexpr bool kSplitLike = PREC == RR_PREC_SPLIT_BF16 || kGram;
    // the split form carries a stage's bitmask words and first B fragments from the stage before
    // it (the Gram form's epilogue leaves no registers for them: it reads them per stage)
    constexpr bool kCarry = PREC == RR_PREC_SPLIT_BF16;
    constexpr int PL = planes_for(PREC);
    constexpr int RECU4 = 64 * PL;                         // uint4 per operand record
    constexpr int REC = kKStage * CB * PL;                 // 1 KB plane records per stage
    constexpr int STAGE_U4 = REC * 64;
    static_assert(REC % NW == 0, "each wave loads the same number of plane records");
    extern __shared__ uint4 smem4[];
    uint4* sA = smem4;                                     // [2][kKStage][CB][PL planes][64 lanes]
    uint32_t* sbits = reinterpret_cast<uint32_t*>(smem4 + 2 * STAGE_U4);   // [TILE][WSTR]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, j = lane & 31;
    // A single pool's contraction is the longer of the two co-resident kernels: its waves
    // issue ahead of the generation waves sharing the SIMD.  (In the batched graph the raised
    // priority measured slower, so batched launches keep the default.)
    if constexpr (!BATCH) __builtin_amdgcn_s_setprio(3);
    // Batched launches walk the (problem, tile) list of all pools; the list is ordered
    // longest problem first, so the grid-stride assignment balances uneven problems, and the
    // workgroups of one XCD take neighbouring tiles of each stride window, so that an XCD's
    // L2 holds the operands of a few pools rather than of every pool in flight.
    const uint64_t ntiles = BATCH ? (uint64_t)a0.nprob * a0.tpp : (a0.num + TILE - 1) / TILE;

    for (uint64_t t = BATCH ? xcd_slot(blockIdx.x, gridDim.x) : blockIdx.x; t < ntiles; t += gridDim.x) {
        const ContractArgs& a = BATCH ? a0.tab[t / a0.tpp] : a0;
        const uint64_t tile0 = (BATCH ? t % a0.tpp : t) * TILE;
        const int nchunks = a.ncb / CB;
        const int nst = a.ks / kKStage;          // ks is a multiple of kKStage
        const int total = nchunks * nst;

        // Stage (chunk, K stage) goes straight from global memory to LDS buffer `buf`; wave w
        // moves plane records w, w + NW, ... (64 lanes x 16 B each).  The records' offsets
        // within a stage are fixed per tile; a stage adds one wave-uniform base.
        constexpr int NREC = REC / NW;
        const int wv = uniform_int(wave);
        uint32_t roff[NREC];
#pragma unroll
        for (int i = 0; i < NREC; ++i) {
            const int r = wv + i * NW;
            const int kk = r / (CB * PL), cb = (r / PL) % CB, p = r % PL;
            roff[i] = (uint32_t)(((kk * a.ncb + cb) * RECU4 + 64 * p + lane) * sizeof(uint4));
        }
        // The copies are buffer loads into LDS over a resource based at the stage: their
        // per-lane byte offsets stay below kKStage ncb records (the host keeps that under 2^31).
        const int ncb_u = uniform_int(a.ncb);
        const uint4* const op_u = uniform_ptr(a.op);
        const uint32_t stage_bytes = (uint32_t)(((kKStage - 1) * ncb_u + CB) * RECU4 * sizeof(uint4));
        auto issue_stage = [&](int chunk, int kst, int buf) {
            const uint4* base = op_u + ((size_t)kst * kKStage * ncb_u + (size_t)chunk * CB) * RECU4;
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)stage_bytes, kBufferWord3);
#pragma unroll
            for (int i = 0; i < NREC; ++i) {
                const lds_ptr_t dst = (lds_ptr_t)(sA + buf * STAGE_U4 + (wv + i * NW) * 64);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, dst, 16, (int)roff[i], 0, 0, 0);
            }
        };
        if (tile0 >= a.num) continue;
        for (int e = tid; e < TILE * 8 * S; e += NW * 64) {
            const int dr = e / (8 * S), w = e % (8 * S);
            const uint64_t idx = tile0 + dr;
            sbits[dr * WSTR + w] = idx < a.num ? __builtin_nontemporal_load(a.bits + idx * (8 * S) + w) : 0u;
        }
        issue_stage(0, 0, 0);
        if (kEarly && total > 1) issue_stage(nst > 1 ? 0 : 1, nst > 1 ? 1 : 0, 1);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        // before the last K step of stage gs: the copy of stage gs + 1 has landed for every wave,
        // and no wave reads buffer gs & 1 any more (the last step's operands are in registers)
        auto early_barrier = [&]() {
            __builtin_amdgcn_sched_barrier(0);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            __builtin_amdgcn_sched_barrier(0);
        };

        float ss[DB], ssa[DB];
#pragma unroll
        for (int db = 0; db < DB; ++db) ss[db] = ssa[db] = 0.f;
        using AccT = std::conditional_t<PREC == RR_PREC_FIXED_I8, i32x16, f32x16>;
        AccT acc[CB][DB];
        const uint32_t* myb = sbits + (wave * 32 * DB + j) * WSTR;

        // (chunk, K stage) of the stage being computed and of the stage two ahead, advanced by one
        // stage per iteration
        int chunk = 0, kst = 0;
        int chunk2 = nst > 2 ? 0 : (nst == 2 ? 1 : 2), kst2 = nst > 2 ? 2 : 0;
        // split forms: A fragments of the step about to run, carried across stages
        bf16x8 Acur[CB][2];
        if constexpr (kSplitLike) {
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int p = 0; p < 2; ++p) Acur[cb][p] = __builtin_bit_cast(bf16x8, sA[(cb * 2 + p) * 64 + lane]);
        }
        // split forms: B dwords of K step kk from bitmask words rotated right by 4 h (lane half h)
        auto expand_w = [&](const uint32_t (&w)[DB][kKStage / 2], int kk, int db) {
            const uint32_t x = w[db][kk >> 1];
            uint4 r;
            if (kk & 1) {
                r = make_uint4(wdword_split<1, 0>(x), wdword_split<1, 1>(x), wdword_split<1, 2>(x),
                               wdword_split<1, 3>(x));
            } else {
                r = make_uint4(wdword_split<0, 0>(x), wdword_split<0, 1>(x), wdword_split<0, 2>(x),
                               wdword_split<0, 3>(x));
            }
            return __builtin_bit_cast(bf16x8, r);
        };
        auto rotated_words = [&](int ks, uint32_t (&w)[DB][kKStage / 2]) {
#pragma unroll
            for (int db = 0; db < DB; ++db)
#pragma unroll
                for (int q = 0; q < kKStage / 2; ++q) {
                    const uint32_t x = myb[32 * db * WSTR + (kKStage / 2) * ks + q];
                    w[db][q] = __builtin_amdgcn_alignbit(x, x, 4 * h);
                }
        };
        // split form: rotated words of the stage about to run and the B fragments of its first
        // step, carried across stages (the last step of a stage prepares the next stage's)
        uint32_t wrc[DB][kKStage / 2];
        bf16x8 Bcc[DB];
        if constexpr (kCarry) {
            rotated_words(0, wrc);
#pragma unroll
            for (int db = 0; db < DB; ++db) Bcc[db] = expand_w(wrc, 0, db);
        }
        for (int gs = 0; gs < total; ++gs) {
            if (kst == 0) {
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                    for (int db = 0; db < DB; ++db)
#pragma unroll
                        for (int e = 0; e < 16; ++e) acc[cb][db][e] = 0;
            }
            if (!kEarly && gs + 1 < total) issue_stage(kst + 1 < nst ? chunk : chunk + 1, kst + 1 < nst ? kst + 1 : 0, (gs + 1) & 1);
            const uint4* st = sA + (gs & 1) * STAGE_U4;
            // bitmask words of this stage: units 128 kst .. 128 kst + 127
            uint32_t wd[DB][kKStage / 2];
            if constexpr (!kSplitLike) {
#pragma unroll
                for (int db = 0; db < DB; ++db)
#pragma unroll
                    for (int q = 0; q < kKStage / 2; ++q) wd[db][q] = myb[32 * db * WSTR + (kKStage / 2) * kst + q];
            }
            if constexpr (kSplitLike) {
                // Software pipeline: the B fragments of step kk + 1 are expanded between the
                // MFMA groups of step kk (scheduling groups place half an expansion after each
                // MFMA); with the carry, the last step expands the next stage's first fragments
                // from its words, read in the middle of the stage.
                uint32_t wr[DB][kKStage / 2], wrn[DB][kKStage / 2];
                bf16x8 Bc[DB], Bn[DB];
                if constexpr (kCarry) {
#pragma unroll
                    for (int db = 0; db < DB; ++db) {
                        Bc[db] = Bcc[db];
#pragma unroll
                        for (int q = 0; q < kKStage / 2; ++q) wr[db][q] = wrc[db][q];
                    }
                } else {
                    rotated_words(kst, wr);
#pragma unroll
                    for (int db = 0; db < DB; ++db) Bc[db] = expand_w(wr, 0, db);
                }
                const int kstn = kst + 1 < nst ? kst + 1 : 0;   // the next stage's (after a tile's last: unused)
                // The A fragments of step kk + 1 are read during step kk, one per MFMA group; those
                // of the next stage's first step are read in the last step, after the barrier that
                // makes that stage's buffer complete (after a tile's last stage the read is of a
                // stale buffer and unused).
                const uint4* stn = sA + ((gs + 1) & 1) * STAGE_U4;
#pragma unroll
                for (int kk = 0; kk < kKStage; ++kk) {
                    const bool more = kk + 1 < kKStage;
                    const bool expand_next = more || kCarry;
                    if (kk == kKStage - 1) early_barrier();
                    if (kCarry && kk == 2) rotated_words(kstn, wrn);
                    bf16x8 An[CB][2];
#pragma unroll
                    for (int g = 0; g < 2 * CB; ++g) {
                        const int cb = g >> 1, p = g & 1;
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int db = 0; db < DB; ++db)
                            acc[cb][db] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Acur[cb][p], Bc[db], acc[cb][db], 0, 0, 0);
                        if (more)
                            An[cb][p] = __builtin_bit_cast(bf16x8, st[(((kk + 1) * CB + cb) * 2 + p) * 64 + lane]);
                        else
                            An[cb][p] = __builtin_bit_cast(bf16x8, stn[(cb * 2 + p) * 64 + lane]);
                        if (expand_next && g < DB) {
                            Bn[g] = more ? expand_w(wr, kk + 1, g) : expand_w(wrn, 0, g);
                            // each MFMA followed by half of the expansion, then the read
#pragma unroll
                            for (int db = 0; db < DB; ++db) {
                                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                                __builtin_amdgcn_sched_group_barrier(0x002, 8 / DB, 0);
                            }
                            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                        } else {
                            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
                            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                            __builtin_amdgcn_sched_group_barrier(0x008, DB - 1, 0);
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                        for (int p = 0; p < 2; ++p) Acur[cb][p] = An[cb][p];
                    if (expand_next) {
#pragma unroll
                        for (int db = 0; db < DB; ++db) Bc[db] = Bn[db];
                    }
                }
                if constexpr (kCarry) {
#pragma unroll
                    for (int db = 0; db < DB; ++db) {
                        Bcc[db] = Bc[db];
#pragma unroll
                        for (int q = 0; q < kKStage / 2; ++q) wrc[db][q] = wrn[db][q];
                    }
                }
            } else if constexpr (PREC == RR_PREC_FIXED_I8) {
                // As the split form with one plane: per K step one int8 MFMA per block pair.
                auto expand = [&](int kk, int db) {
                    const uint32_t w = wd[db][kk >> 1];
                    return __builtin_bit_cast(i32x4, expand_i8((w >> (16 * (kk & 1) + 8 * h)) & 0xFFu));
                };
                i32x4 Bc[DB], Bn[DB];
#pragma unroll
                for (int db = 0; db < DB; ++db) Bc[db] = expand(0, db);
#pragma unroll
                for (int kk = 0; kk < kKStage; ++kk) {
                    const bool more = kk + 1 < kKStage;
                    i32x4 A[CB];
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) A[cb] = __builtin_bit_cast(i32x4, st[(kk * CB + cb) * 64 + lane]);
                    if (kk == kKStage - 1) early_barrier();
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int db = 0; db < DB; ++db)
                            acc[cb][db] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[cb], Bc[db], acc[cb][db], 0, 0, 0);
                        __builtin_amdgcn_sched_barrier(0);
                        if (more && cb < DB) Bn[cb] = expand(kk + 1, cb);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    if (more) {
#pragma unroll
                        for (int db = 0; db < DB; ++db) Bc[db] = Bn[db];
                    }
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < kKStage; ++kk) {
                    {
#pragma unroll
                        for (int cb = 0; cb < CB; ++cb) {
                            f32x16 stp[DB];
#pragma unroll
                            for (int db = 0; db < DB; ++db)
#pragma unroll
                                for (int e = 0; e < 16; ++e) stp[db][e] = 0.f;
#pragma unroll
                            for (int p = 0; p < 2; ++p) {
                                const uint4 av = st[((kk * CB + cb) * 2 + p) * 64 + lane];
                                const float af[4] = {__uint_as_float(av.x), __uint_as_float(av.y),
                                                     __uint_as_float(av.z), __uint_as_float(av.w)};
#pragma unroll
                                for (int q = 0; q < 4; ++q) {
#pragma unroll
                                    for (int db = 0; db < DB; ++db) {
                                        const uint32_t w = wd[db][kk >> 1];
                                        const float bv = (float)((w >> (16 * (kk & 1) + 8 * p + 2 * q + h)) & 1u);
                                        stp[db] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[q], bv, stp[db], 0, 0, 0);
                                    }
                                }
                            }
#pragma unroll
                            for (int db = 0; db < DB; ++db) acc[cb][db] += stp[db];
                        }
                    }
                }
            }
            if (kEarly && gs + 2 < total) issue_stage(chunk2, kst2, gs & 1);   // buffer gs & 1 is free
            if (kst == nst - 1) {
                // ||G||^2 over this chunk's covariates
#pragma unroll
                for (int db = 0; db < DB; ++db) {
                    float s2 = 0.f, sa = 0.f;
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb) {
                        if constexpr (kGram) {
                            // rows 8 (r / 4) + 4h + r % 4 of unit block chunk CB + cb: one
                            // bitmask word of this lane's draw
                            const uint32_t wb = myb[32 * db * WSTR + chunk * CB + cb];
#pragma unroll
                            for (int r = 0; r < 16; ++r) {
                                const bool t = (wb >> (8 * (r / 4) + 4 * h + (r % 4))) & 1u;
                                const float v = acc[cb][db][r];
                                s2 += t ? v : 0.f;
                                sa += t ? fabsf(v) : 0.f;
                            }
                        } else if constexpr (PREC == RR_PREC_FIXED_I8) {
                            // G = s I, I the exact int32 sums of this block
                            float t = 0.f;
                            const float sc = a.bscale[chunk * CB + cb];
                            if (a.maxmode) {
#pragma unroll
                                for (int r = 0; r < 16; ++r) {
                                    const float g = (float)acc[cb][db][r];
                                    t = fmaxf(t, g * g);
                                }
                                s2 = fmaxf(s2, (sc * sc) * t);
                            } else {
#pragma unroll
                                for (int r = 0; r < 16; ++r) {
                                    const float g = (float)acc[cb][db][r];
                                    t = fmaf(g, g, t);
                                }
                                s2 = fmaf(sc * sc, t, s2);
                            }
                        } else {
                            if (a.maxmode) {
#pragma unroll
                                for (int r = 0; r < 16; ++r) s2 = fmaxf(s2, acc[cb][db][r] * acc[cb][db][r]);
                            } else {
#pragma unroll
                                for (int r = 0; r < 16; ++r) s2 = fmaf(acc[cb][db][r], acc[cb][db][r], s2);
                            }
                        }
                    }
                    // per-column criterion: the largest G_j^2 instead of the sum
                    ss[db] = (!kGram && a.maxmode) ? fmaxf(ss[db], s2) : ss[db] + s2;
                    if constexpr (kGram) ssa[db] += sa;
                }
            }
            if constexpr (!kEarly) {
                __builtin_amdgcn_s_waitcnt(0);     // this wave's loads of the next stage landed
                __syncthreads();
            }
            if (++kst == nst) {
                kst = 0;
                ++chunk;
            }
            if (++kst2 == nst) {
                kst2 = 0;
                ++chunk2;
            }
        }
        if constexpr (kEarly) __syncthreads();   // every wave done with this tile's LDS before the next tile's

#pragma unroll
        for (int db = 0; db < DB; ++db) {
            // the split form summed (2G)^2, the Gram form 2 G' (W enters as 2.0)
            const float other = __shfl_xor(ss[db], 32, 64);
            const float s2 = ((!kGram && a.maxmode) ? fmaxf(ss[db], other) : ss[db] + other) *
                             (PREC == RR_PREC_SPLIT_BF16 ? 0.25f : (kGram ? 0.5f : 1.0f));
            const uint64_t idx = tile0 + wave * 32 * DB + 32 * db + j;
            const bool live = h == 0 && idx < a.num;
            float m32, err;
            if constexpr (kGram) {
                // M >= 0: clamping a rounded negative sum keeps the bound and the key order
                const float sa = (ssa[db] + __shfl_xor(ssa[db], 32, 64)) * 0.5f;
                m32 = fmaxf(a.scale * s2, 0.0f);
                err = a.safety * (a.scale * (a.csq + a.gamma_ss * sa));
            } else {
                // sum_j |G_j| cabs_j <= ||G|| ||cabs|| (Cauchy-Schwarz); cnorm = ||cabs|| (1 + 2^-20)
                const float s1 = sqrtf(s2) * (1.0f + 0x1p-20f) * a.cnorm;
                m32 = a.scale * s2;
                err = a.safety * (a.scale * (a.two_kappa * s1 + a.csq) + a.gamma_ss * m32);
            }
            const float hi = (m32 + err) * (1.0f + 0x1p-21f);
            const float lo = fmaxf((m32 - err) * (1.0f - 0x1p-21f), 0.0f);
            if (a.out_err) {
                if (live) {
                    a.out_m32[idx] = m32;
                    a.out_err[idx] = err;
                }
            } else if (a.out_hi) {
                if (live) {
                    a.out_hi[idx] = hi;
                    a.out_lo[idx] = lo;
                    a.out_m32[idx] = m32;
                }
            } else {
                const bool pass = live && (a.U == nullptr || lo <= *a.U);
                const uint64_t bm = __ballot(pass);
                if (bm) {
                    const int first = (int)__builtin_ctzll(bm);
                    uint32_t base = 0;
                    if (lane == first) base = atomicAdd(a.cand_count, (uint32_t)__builtin_popcountll(bm));
                    base = __shfl(base, first, 64);
                    if (pass) {
                        const uint32_t pos = base + __builtin_amdgcn_mbcnt_hi(
                                                        (uint32_t)(bm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bm, 0u));
                        if (pos < a.cand_cap) {
                            a.cand_key[pos] = a.keylist ? a.keylist[idx] : a.key_begin + idx;
                            a.cand_hi[pos] = hi;
                            a.cand_lo[pos] = lo;
                            a.cand_m[pos] = m32;
                        }
                    }
                }
            }
        }
    }
}

// Tile shapes: covariate blocks per chunk (CB) and 32-draw blocks per wave (DB).  Split
// BF16: 8 waves (two per SIMD, so one wave's bit expansion on the VALU overlaps the other's
// MFMA), each with 2 x DB accumulator blocks of 32x32 (<= 168 registers, leaving room for
// three generation waves per SIMD); fixed I8: the same shape with one operand plane (half
// the LDS stage); FP32: 4 waves of 2 x DB blocks plus a per-K-step block set.  The default DB is 2 where the tile's bitmasks fit in LDS beside the operand stages;
// the autotuner may pick 1.  Per-draw arithmetic (and so every M32) does not depend on NW
// or DB, only on CB.
constexpr int kCB = 2;
constexpr bool mfma16(int prec) {
    return prec == RR_PREC_SPLIT_BF16 || prec == RR_PREC_FIXED_I8 || prec == RR_PREC_GRAM_BF16;
}
constexpr int nw_for(int prec, int S) { return mfma16(prec) && S <= 8 ? 8 : 4; }
constexpr size_t lds_for(int prec, int S, int db) {
    return sizeof(uint4) * 2 * kKStage * kCB * 64 * planes_for(prec) +
           sizeof(uint32_t) * (nw_for(prec, S) * 32 * db) * (8 * S + 1);
}
constexpr size_t kMaxLds = 160 * 1024;
constexpr int db_default(int prec, int S) {
    return mfma16(prec) ? (S <= 4 ? 2 : 1) : (S <= 8 ? 2 : 1);
}

template <int PREC, int S, int DB, bool BATCH>
static hipError_t launch_contract_t(const ContractArgs& a, int grid, hipStream_t st) {
    if constexpr (lds_for(PREC, S, DB) > kMaxLds) {
        return hipErrorInvalidConfiguration;
    } else {
        auto k = contract_kernel<PREC, nw_for(PREC, S), kCB, DB, S, BATCH>;
        const size_t lds = lds_for(PREC, S, DB);
        hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, dim3(grid), dim3(64 * nw_for(PREC, S)), lds, st, a);
        return hipGetLastError();
    }
}

template <int PREC, bool BATCH>
static hipError_t launch_contract_p(int S, int db, const ContractArgs& a, int grid, hipStream_t st) {
#define RR_CASE(SV)                                                                       \
    case SV:                                                                              \
        return db == 1 ? launch_contract_t<PREC, SV, 1, BATCH>(a, grid, st)               \
                       : launch_contract_t<PREC, SV, 2, BATCH>(a, grid, st);
    switch (S) {
        RR_CASE(1)
        RR_CASE(2)
        RR_CASE(4)
        RR_CASE(8)
        RR_CASE(16)
    }
#undef RR_CASE
    return hipErrorInvalidValue;
}

bool contract_db_ok(int prec, int S, int db) {
    return (db == 1 || db == 2) && lds_for(prec, S, db) <= kMaxLds;
}
int contract_db_default(int prec, int S) { return db_default(prec, S); }

// db = 0 selects the default tile.  Batched launches take the problem table from a.tab.
hipError_t launch_contract(int S, int prec, int db, bool batch, const ContractArgs& a, int grid, hipStream_t st) {
    grid = std::max(1, grid);
    if (db == 0) db = db_default(prec, S);
    if (!contract_db_ok(prec, S, db)) return hipErrorInvalidConfiguration;
    if (prec == RR_PREC_SPLIT_BF16)
        return batch ? launch_contract_p<RR_PREC_SPLIT_BF16, true>(S, db, a, grid, st)
                     : launch_contract_p<RR_PREC_SPLIT_BF16, false>(S, db, a, grid, st);
    if (prec == RR_PREC_FIXED_I8)
        return batch ? launch_contract_p<RR_PREC_FIXED_I8, true>(S, db, a, grid, st)
                     : launch_contract_p<RR_PREC_FIXED_I8, false>(S, db, a, grid, st);
    if (prec == RR_PREC_GRAM_BF16)
        return batch ? launch_contract_p<RR_PREC_GRAM_BF16, true>(S, db, a, grid, st)
                     : launch_contract_p<RR_PREC_GRAM_BF16, false>(S, db, a, grid, st);
    return batch ? launch_contract_p<RR_PREC_FP32, true>(S, db, a, grid, st)
                 : launch_contract_p<RR_PREC_FP32, false>(S, db, a, grid, st);
}

// Vector registers per lane and waves per workgroup of a contraction tile (0 if unknown).
template <int PREC, int S, int DB, bool BATCH>
static int contract_vgprs_t() {
    if constexpr (lds_for(PREC, S, DB) > kMaxLds) {
        return 0;
    } else {
        hipFuncAttributes fa{};
        auto k = contract_kernel<PREC, nw_for(PREC, S), kCB, DB, S, BATCH>;
        return hipFuncGetAttributes(&fa, (const void*)k) == hipSuccess ? fa.numRegs : 0;
    }
}

template <int PREC, bool BATCH>
static int contract_vgprs_p(int S, int db) {
    switch (S) {
#define RR_CASE(SV) \
    case SV: return db == 1 ? contract_vgprs_t<PREC, SV, 1, BATCH>() : contract_vgprs_t<PREC, SV, 2, BATCH>();
        RR_CASE(1)
        RR_CASE(2)
        RR_CASE(4)
        RR_CASE(8)
        RR_CASE(16)
#undef RR_CASE
    }
    return 0;
}

int contract_kernel_vgprs(int prec, int S, int db, bool batch) {
    if (db == 0) db = db_default(prec, S);
    if (!contract_db_ok(prec, S, db)) return 0;
    if (prec == RR_PREC_SPLIT_BF16)
        return batch ? contract_vgprs_p<RR_PREC_SPLIT_BF16, true>(S, db) : contract_vgprs_p<RR_PREC_SPLIT_BF16, false>(S, db);
    if (prec == RR_PREC_FIXED_I8)
        return batch ? contract_vgprs_p<RR_PREC_FIXED_I8, true>(S, db) : contract_vgprs_p<RR_PREC_FIXED_I8, false>(S, db);
    if (prec == RR_PREC_GRAM_BF16)
        return batch ? contract_vgprs_p<RR_PREC_GRAM_BF16, true>(S, db) : contract_vgprs_p<RR_PREC_GRAM_BF16, false>(S, db);
    return batch ? contract_vgprs_p<RR_PREC_FP32, true>(S, db) : contract_vgprs_p<RR_PREC_FP32, false>(S, db);
}
int contract_waves(int prec, int S) { return nw_for(prec, S); }

int contract_tile(int prec, int S, int db) {
    if (db == 0) db = db_default(prec, S);
    return nw_for(prec, S) * 32 * db;
}
int draw_cb(int, int) { return kCB; }

}  // namespace rr
