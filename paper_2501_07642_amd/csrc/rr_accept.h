// Acceptance pieces shared by the single-pool and batched pipelines (device code).
//
// Rules (section 2.2; Appendix A part C): threshold, M <= a; q-quantile, the
// k = ceil(q N (1 - 1e-12)) smallest M, with values within a relative eps = 1e-10 of the
// k-th smallest taken in key order.  Every draw carries FP32 bounds [lo, hi] around its
// FP64 value; with T_lo / T_hi the k-th smallest lo / hi, a draw with hi < T_lo (1 - eps) is
// accepted outright, one with lo > T_hi (1 + eps) is rejected outright, and the rest (the
// guard band) are decided on their FP64 recomputation.
#pragma once

#include "rr_internal.h"

namespace rr {

constexpr double kEpsTie = 1e-10;
constexpr double kQFuzz = 1e-12;

// Classification of one draw from its FP32 bounds (both modes).  Quantile cuts are
// lo_cut = T_lo (1 - eps), hi_cut = T_hi (1 + eps), evaluated in FP64.
__device__ __forceinline__ void classify_one(double hi, double lo, int mode, double a, double lo_cut,
                                             double hi_cut, bool* acc, bool* band) {
    if (mode == RR_MODE_QUANTILE) {
        *acc = hi < lo_cut;
        *band = !*acc && lo <= hi_cut && hi >= lo_cut;
    } else {
        *acc = hi <= a;
        *band = !*acc && lo <= a;
    }
}

// One wave finds the bin of a 256-bin histogram holding the need-th smallest entry (1-based):
// bin and the count below it, broadcast to every lane; false when the histogram holds fewer
// than need entries.
__device__ inline bool wave_digit_select(const uint32_t* hist, uint32_t need, uint32_t* bin, uint32_t* below) {
    const int lane = lane_id();
    const uint4 c = reinterpret_cast<const uint4*>(hist)[lane];
    const uint32_t tot = c.x + c.y + c.z + c.w;
    uint32_t run = wave_incl_scan(tot) - tot;
    const uint32_t cc[4] = {c.x, c.y, c.z, c.w};
    int hit = -1;
    uint32_t cb = 0;
    for (int j = 0; j < 4; ++j) {
        if (hit < 0 && run < need && need <= run + cc[j]) {
            hit = j;
            cb = run;
        }
        run += cc[j];
    }
    const uint64_t m = __ballot(hit >= 0);
    if (m == 0) return false;
    const int src = (int)__builtin_ctzll(m);
    *bin = (uint32_t)__shfl(4 * lane + hit, src, 64);
    *below = __shfl(cb, src, 64);
    return true;
}

// k-th smallest (1-based) of v[i] over i < n with ok[i] (ok null = all), by one workgroup:
// eight 8-bit radix passes with an LDS histogram `hist` of 256 bins.
__device__ inline uint64_t block_select_u64(const uint64_t* v, const uint8_t* ok, uint32_t n, uint32_t k,
                                            uint32_t* hist) {
    __shared__ uint32_t s_bin, s_below;
    uint64_t prefix = 0;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
        __syncthreads();
        const uint64_t m = shift == 56 ? 0ull : (~0ull << (shift + 8));
        for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
            if (ok && !ok[i]) continue;
            const uint64_t x = v[i];
            if ((x & m) == (prefix & m)) atomicAdd(&hist[(x >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t run = 0;
            int bin = 255;
            for (int b = 0; b < 256; ++b) {
                if (run + hist[b] >= k) {
                    bin = b;
                    break;
                }
                run += hist[b];
            }
            s_bin = (uint32_t)bin;
            s_below = run;
        }
        __syncthreads();
        prefix |= (uint64_t)s_bin << shift;
        k -= s_below;
        __syncthreads();
    }
    return prefix;
}

// Final acceptance among the guard band (FP64 values bm of keys bkey, nb = st->band_count
// entries), by one workgroup; `work` holds nb bytes of scratch.  Threshold: bm <= a.
// Quantile: need = k - nL band members are accepted: those below t (1 - eps), t the need-th
// smallest band value, then the smallest keys among the values within eps t of t.
__device__ inline void band_accept_block(const uint64_t* bkey, const double* bm, uint8_t* work, AcceptState* st,
                                         int mode, double a, uint64_t* acc_key, double* acc_m, uint8_t* acc_flag,
                                         uint32_t acc_cap, uint32_t* hist) {
    __shared__ uint32_t s_cnt;
    const uint32_t nb = st->band_count;
    if (mode == RR_MODE_THRESHOLD) {
        for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) {
            if (bm[i] <= a) {
                const uint32_t p = atomicAdd(&st->acc_count, 1u);
                if (p < acc_cap) {
                    acc_key[p] = bkey[i];
                    acc_m[p] = bm[i];
                    if (acc_flag) acc_flag[p] = 1;
                }
            }
        }
        return;
    }
    const int64_t need = (int64_t)st->k - (int64_t)st->nL;
    if (need < 1 || (int64_t)nb < need) {
        if (threadIdx.x == 0) st->guard_fail = 1;
        return;
    }
    const uint64_t* bits = reinterpret_cast<const uint64_t*>(bm);
    const double t = __longlong_as_double((long long)block_select_u64(bits, nullptr, nb, (uint32_t)need, hist));
    const double lo_cut = t * (1.0 - kEpsTie), tol = kEpsTie * t;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) {
        const bool low = bm[i] < lo_cut;
        const bool near = fabs(bm[i] - t) <= tol;
        work[i] = near ? 1 : 0;
        if (low) atomicAdd(&s_cnt, 1u);
    }
    __syncthreads();
    const int64_t take = need - (int64_t)s_cnt;
    uint64_t kstar = 0;
    if (take >= 1) kstar = block_select_u64(bkey, work, nb, (uint32_t)take, hist);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) {
        const bool low = bm[i] < lo_cut;
        const bool pick = low || (work[i] && take >= 1 && bkey[i] <= kstar);
        if (pick) {
            const uint32_t p = atomicAdd(&st->acc_count, 1u);
            if (p < acc_cap) {
                acc_key[p] = bkey[i];
                acc_m[p] = bm[i];
                if (acc_flag) acc_flag[p] = 1;
            }
        }
    }
}

// Bitonic sort of CHUNK (key, index) pairs in LDS by (key, index), by one workgroup.
template <int CHUNK>
__device__ inline void bitonic_sort_lds(uint64_t* sk, uint32_t* si) {
    for (int size = 2; size <= CHUNK; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < CHUNK / 2; t += blockDim.x) {
                const int i = 2 * t - (t & (stride - 1));
                const int jx = i + stride;
                const bool up = ((i & size) == 0);
                const uint64_t ki = sk[i], kj = sk[jx];
                const uint32_t ii = si[i], ij = si[jx];
                const bool swap = up ? (ki > kj || (ki == kj && ii > ij)) : (ki < kj || (ki == kj && ii < ij));
                if (swap) {
                    sk[i] = kj;
                    sk[jx] = ki;
                    si[i] = ij;
                    si[jx] = ii;
                }
            }
            __syncthreads();
        }
    }
}

}  // namespace rr
