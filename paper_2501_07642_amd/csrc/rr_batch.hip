// Batched pools: many independent Monte Carlo pools of uneven n and d in one graph launch
// (section 2.1 "Batched processing"; section 2.3 generate_randomizations per pool).
//
// Work list.  Pools are grouped by S (256-unit chunks per draw, which fixes the bitmask
// layout and the kernel instantiation) and, inside a group, ordered by MFMA work per draw
// (ks x ncb), largest first.  Draws are processed in rounds of up to C draws per pool (C
// bounds the bitmask buffers; the first and the last round are about C / 4, since nothing
// overlaps them); in every round, for every group, a persistent generation launch walks the
// (pool, draw) list and a persistent contraction launch walks the (pool, tile) list, the
// generation of the next group / round overlapping the contraction of the current one on a
// second stream.  The contraction writes, per draw, the FP32 bounds [lo, hi] and m32
// densely.  Then one workgroup per pool selects T_lo / T_hi (radix select in LDS) and
// classifies its draws, the guard bands of all pools are recomputed in FP64 (one launch per
// group), and one workgroup per pool applies the final rule, sorts its accepted keys in LDS
// and writes the caller's outputs.
//
// The whole sequence is captured once into a hipGraph (no memset nodes: state is cleared by
// a kernel) and replayed while the call's arguments stay the same.  Results equal those of
// rr_draw_balance on every pool: the same kernels compute every per-draw value, and the
// selection rules are the same.  A pool whose guard band exceeds the batched capacity is
// rerun through the single-pool pipeline.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "rr_accept.h"
#include "rr_internal.h"

namespace rr {

constexpr int kFinishSort = 2048;              // accepted keys sorted in LDS per pool
constexpr uint32_t kBatchBandCap = 1u << 14;   // guard-band entries per pool (d < n - 1)
// Bytes per bitmask round buffer.  It sets the round length C: the contraction stream trails
// the generation stream by one (group, round) item, so shorter rounds start and end the
// overlap sooner; 512 MB (about 21 rounds over the 512-pool workload) measured 3% faster
// than 1 GB, and 256 MB slower again from the kernel count.
constexpr size_t kBitsBudget = size_t(1) << 29;
// Recheck workgroups per CU: the bands of a bitmask class (up to kBatchBandCap entries per
// pool; up to every draw where d >= n - 1, since there M hardly varies across draws under a
// small ridge and most draws sit within the error bound of the boundary) form one flat list
// of tiles that this many workgroups per CU stride over.
constexpr int kBatchRecheckWgsPerCu = 2;

// Per-pool record of the acceptance stages (device).
struct PoolRec {
    const float* hi;
    const float* lo;
    const float* m;
    uint64_t key_begin;
    uint64_t* acc_key;
    double* acc_m;
    uint32_t acc_cap;
    uint64_t* band_key;
    double* band_m;
    uint8_t* band_work;
    uint32_t band_cap;
    AcceptState* st;
    uint64_t* out_key;
    double* out_m;
    uint64_t capacity;
    double a;             // threshold modes: the pool's threshold
};

__global__ void batch_init_kernel(AcceptState* st, int nprob, uint32_t k) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob) {
        AcceptState s{};
        s.k = k;
        st[p] = s;
    }
}

// One workgroup per pool: T_hi / T_lo by radix select over the pool's N draws (quantile
// mode), then outright acceptances and guard-band members.
__global__ __launch_bounds__(1024) void batch_select_kernel(const PoolRec* recs, uint32_t N, int mode) {
    __shared__ uint32_t hist[2][256];
    __shared__ uint32_t s_prefix[2], s_krem[2], s_fail, s_acc, s_band;
    const PoolRec& r = recs[blockIdx.x];
    const int tid = threadIdx.x, wave = tid >> 6;
    double lo_cut = 0.0, hi_cut = 0.0;
    if (tid == 0) {
        s_fail = 0;
        s_acc = 0;
        s_band = 0;
    }
    if (mode == RR_MODE_QUANTILE) {
        if (tid < 2) {
            s_prefix[tid] = 0;
            s_krem[tid] = r.st->k;
        }
        for (int shift = 24; shift >= 0; shift -= 8) {
            for (int i = tid; i < 512; i += blockDim.x) (&hist[0][0])[i] = 0;
            __syncthreads();
            const uint32_t m = shift == 24 ? 0u : (0xFFFFFFFFu << (shift + 8));
            const uint32_t p0 = s_prefix[0] & m, p1 = s_prefix[1] & m;
            for (uint32_t i = tid; i < N; i += blockDim.x) {
                const uint32_t x0 = __float_as_uint(r.hi[i]);
                const uint32_t x1 = __float_as_uint(r.lo[i]);
                if ((x0 & m) == p0) atomicAdd(&hist[0][(x0 >> shift) & 255u], 1u);
                if ((x1 & m) == p1) atomicAdd(&hist[1][(x1 >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (wave < 2) {
                uint32_t bin, below;
                const bool ok = wave_digit_select(hist[wave], s_krem[wave], &bin, &below);
                if (lane_id() == 0) {
                    if (!ok) {
                        s_fail = 1;
                    } else {
                        s_prefix[wave] |= bin << shift;
                        s_krem[wave] -= below;
                    }
                }
            }
            __syncthreads();
        }
        if (s_fail) {
            if (tid == 0) r.st->guard_fail = 1;
            return;
        }
        lo_cut = (double)__uint_as_float(s_prefix[1]) * (1.0 - kEpsTie);
        hi_cut = (double)__uint_as_float(s_prefix[0]) * (1.0 + kEpsTie);
    }
    __syncthreads();
    for (uint32_t i = tid; i < N; i += blockDim.x) {
        bool acc, band;
        classify_one(r.hi[i], r.lo[i], mode, r.a, lo_cut, hi_cut, &acc, &band);
        if (acc) {
            const uint32_t p = atomicAdd(&s_acc, 1u);
            if (p < r.acc_cap) {
                r.acc_key[p] = r.key_begin + i;
                r.acc_m[p] = (double)r.m[i];
            }
        } else if (band) {
            const uint32_t p = atomicAdd(&s_band, 1u);
            if (p < r.band_cap) r.band_key[p] = r.key_begin + i;
        }
    }
    __syncthreads();
    if (tid == 0) {
        r.st->nL = s_acc;
        r.st->acc_count = s_acc;
        r.st->band_count = min(s_band, r.band_cap);
        if (s_band > r.band_cap || s_acc > r.acc_cap) r.st->overflow = 1;
    }
}

// One workgroup per pool: final rule over the rechecked band, then the accepted keys sorted
// in LDS and written with their M to the caller's outputs (when they fit: at most
// kFinishSort keys and the caller's capacity; otherwise the host finishes the pool).
__global__ __launch_bounds__(1024) void batch_finish_kernel(const PoolRec* recs, int mode) {
    __shared__ uint32_t hist[256];
    __shared__ uint64_t sk[kFinishSort];
    __shared__ uint32_t si[kFinishSort];
    __shared__ uint32_t s_K, s_bad;
    const PoolRec& r = recs[blockIdx.x];
    AcceptState* st = r.st;
    if (st->overflow || st->guard_fail) return;   // uniform: written by an earlier kernel
    band_accept_block(r.band_key, r.band_m, r.band_work, st, mode, r.a, r.acc_key, r.acc_m, nullptr, r.acc_cap, hist);
    __syncthreads();
    if (threadIdx.x == 0) {
        // atomics keep these reads at the coherence point the band atomics updated
        s_K = atomicAdd(&st->acc_count, 0u);
        s_bad = atomicOr(&st->guard_fail, 0u);
    }
    __syncthreads();
    const uint32_t K = s_K;
    if (s_bad || K > r.acc_cap || K > r.capacity || K > (uint32_t)kFinishSort) return;
    for (int i = threadIdx.x; i < kFinishSort; i += blockDim.x) {
        sk[i] = (uint32_t)i < K ? r.acc_key[i] : ~0ull;
        si[i] = (uint32_t)i < K ? (uint32_t)i : 0xFFFFFFFFu;
    }
    __syncthreads();
    bitonic_sort_lds<kFinishSort>(sk, si);
    for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) {
        r.out_key[i] = sk[i];
        r.out_m[i] = r.acc_m[si[i]];
    }
    if (threadIdx.x == 0) st->done = 1;
}

// ---------------------------------------------------------------------------------------
// Host side.
struct BatchState {
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t s_main = nullptr, s_gen = nullptr;
    std::vector<hipEvent_t> ev;
    hipEvent_t t0 = nullptr, t1 = nullptr, join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> sig;      // arguments of the captured call
    int64_t kernels = 0;            // kernel launches in the graph
};

void free_batch_state(Problem& P) {
    BatchState* b = P.batch;
    if (!b) return;
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    for (hipEvent_t e : b->ev) hipEventDestroy(e);
    if (b->t0) hipEventDestroy(b->t0);
    if (b->t1) hipEventDestroy(b->t1);
    if (b->join) hipEventDestroy(b->join);
    if (b->s_main) hipStreamDestroy(b->s_main);
    if (b->s_gen) hipStreamDestroy(b->s_gen);
    hipFree(b->ws);
    delete b;
    P.batch = nullptr;
}

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Group {
    int S;
    std::vector<int64_t> idx;   // pools, largest work per draw first
    Tune tune;
    int tile;
    size_t bits_off;            // uint32 words from the start of a round buffer
};

}  // namespace

}  // namespace rr

using namespace rr;

extern "C" rr_status rr_draw_balance_batched(rr_problem* const* P, int64_t nprob, const uint64_t* seeds,
                                             uint64_t key_begin, uint64_t num_draws, int mode, double q_or_a,
                                             int precision, uint64_t* const* d_keys, double* const* d_M,
                                             uint64_t capacity, uint64_t* h_counts, void* stream) {
    const auto t_start = std::chrono::steady_clock::now();
    if (!P || nprob < 0 || (nprob > 0 && (!seeds || !d_keys || !d_M || !h_counts))) {
        set_error("rr_draw_balance_batched: invalid argument");
        return RR_E_ARG;
    }
    if (nprob == 0) return RR_OK;
    const uint64_t N = num_draws;
    if (N == 0 || N > 0xFFFFFFFFull || key_begin + N < key_begin ||
        (mode != RR_MODE_QUANTILE && mode != RR_MODE_THRESHOLD && mode != RR_MODE_CHI2_QUANTILE) ||
        !valid_prec(precision) || nprob > (1 << 20)) {
        set_error("rr_draw_balance_batched: invalid argument");
        return RR_E_ARG;
    }
    int dev = 0;
    RR_HIP(hipGetDevice(&dev));
    for (int64_t i = 0; i < nprob; ++i) {
        if (!P[i] || !d_keys[i] || !d_M[i]) {
            set_error("rr_draw_balance_batched: null handle or output");
            return RR_E_ARG;
        }
        if (P[i]->P.device != dev) {
            set_error("rr_draw_balance_batched: handles must belong to the current device");
            return RR_E_ARG;
        }
    }
    uint64_t k = 0;
    if (mode == RR_MODE_QUANTILE) {
        if (!(q_or_a > 0.0 && q_or_a <= 1.0)) {
            set_error("rr_draw_balance_batched: q must be in (0, 1]");
            return RR_E_ARG;
        }
        k = (uint64_t)std::ceil(q_or_a * (double)N * (1.0 - kQFuzz));
        k = std::min<uint64_t>(std::max<uint64_t>(k, 1), N);
        if (k > capacity) {
            for (int64_t i = 0; i < nprob; ++i) h_counts[i] = k;
            set_error("rr_draw_balance_batched: capacity below the accepted count");
            return RR_E_CAPACITY;
        }
    } else if (mode == RR_MODE_CHI2_QUANTILE) {
        if (!(q_or_a > 0.0 && q_or_a <= 1.0)) {
            set_error("rr_draw_balance_batched: q must be in (0, 1]");
            return RR_E_ARG;
        }
    } else if (std::isnan(q_or_a)) {
        set_error("rr_draw_balance_batched: threshold is NaN");
        return RR_E_ARG;
    }
    // chi-square mode: each pool's threshold c_q of chi^2_d, then threshold acceptance
    const bool chi2 = mode == RR_MODE_CHI2_QUANTILE;
    const double q_in = q_or_a;
    if (chi2) mode = RR_MODE_THRESHOLD;
    hipStream_t st = (hipStream_t)stream;
    Problem& lead = P[0]->P;
    if (!lead.batch) lead.batch = new BatchState();
    BatchState& B = *lead.batch;
    if (!B.s_main) RR_HIP(hipStreamCreateWithFlags(&B.s_main, hipStreamNonBlocking));
    if (!B.s_gen) RR_HIP(hipStreamCreateWithFlags(&B.s_gen, hipStreamNonBlocking));
    if (!B.t0) RR_HIP(hipEventCreate(&B.t0));
    if (!B.t1) RR_HIP(hipEventCreate(&B.t1));
    if (!B.join) RR_HIP(hipEventCreateWithFlags(&B.join, hipEventDisableTiming));
    const int cus = device_cus(dev);
    if (precision == RR_PREC_GRAM_BF16) {
        for (int64_t i = 0; i < nprob; ++i) {
            if (P[i]->P.metric == RR_METRIC_MAX_SMD) {
                set_error("rr_draw_balance_batched: the Gram form has no per-column sums (RR_METRIC_MAX_SMD)");
                return RR_E_ARG;
            }
            const rr_status s = ensure_gram(P[i]->P, st);
            if (s != RR_OK) return s;
        }
    }

    // ---- plan: groups by S, largest work first; default tiles per group
    std::vector<Group> groups;
    for (int S = kMaxS; S >= 1; S >>= 1) {
        Group g{};
        g.S = S;
        for (int64_t i = 0; i < nprob; ++i)
            if (P[i]->P.S == S) g.idx.push_back(i);
        if (g.idx.empty()) continue;
        std::stable_sort(g.idx.begin(), g.idx.end(), [&](int64_t x, int64_t y) {
            return P[x]->P.ks * P[x]->P.ncb > P[y]->P.ks * P[y]->P.ncb;
        });
        // Default tiles to start from, not the single-pool choice: a class's generation and
        // contraction run side by side over many pools, and the choice that is fastest for one
        // pool alone (for S = 4, one draw tile per wave with four generation workgroups per CU)
        // measured about 10% slower in this launch than two tiles with three.  A tune file may
        // hold a per-class choice (read below).
        g.tune = tune_default(precision, S, true);
        g.tile = contract_tile(precision, S, g.tune.db);
        groups.push_back(g);
    }
    size_t words_per_draw = 0;   // bitmask words of one draw index over all pools
    for (Group& g : groups) {
        g.bits_off = words_per_draw;
        words_per_draw += (size_t)g.idx.size() * 8 * g.S;
    }
    uint64_t C = std::max<uint64_t>(512, kBitsBudget / (4 * words_per_draw));
    C = std::min<uint64_t>(C / 512 * 512, N);
    for (Group& g : groups) g.bits_off *= C;
    // Round schedule: the first round's generation runs with no contraction beside it and
    // the last round's contraction with no generation, so both are cut to about C / 4
    // (multiples of 512); the rounds between are C draws each, and none exceeds C.
    std::vector<uint64_t> rbeg, rcnt;
    {
        const uint64_t C0 = std::max<uint64_t>(512, C / 4 / 512 * 512);
        uint64_t at = 0;
        auto push = [&](uint64_t c) {
            rbeg.push_back(at);
            rcnt.push_back(c);
            at += c;
        };
        if (N > 2 * C0) push(C0);
        while (N - at > C + C0) push(C);
        const uint64_t rest = N - at;
        if (rest > C || rest > 2 * C0) {   // rest <= C + C0 here, so rest - C0 <= C
            push(rest - C0);
            push(C0);
        } else if (rest > 0) {
            push(rest);
        }
    }
    const uint64_t R = rbeg.size();
    const uint32_t acc_cap = (uint32_t)(mode == RR_MODE_QUANTILE ? k : std::min<uint64_t>(capacity, N));
    // guard-band capacity per pool, packed back to back
    std::vector<uint32_t> bcap((size_t)nprob);
    std::vector<size_t> boff((size_t)nprob);
    size_t band_total_cap = 0;
    for (int64_t i = 0; i < nprob; ++i) {
        const Problem& Q = P[i]->P;
        bcap[i] = (uint32_t)std::min<uint64_t>(N, Q.d >= Q.n - 1 ? N : kBatchBandCap);
        boff[i] = band_total_cap;
        band_total_cap += bcap[i];
    }

    // ---- workspace
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t np = (size_t)nprob;
    const size_t o_hi = take(4 * np * N), o_lo = take(4 * np * N), o_m = take(4 * np * N);
    const size_t o_bits0 = take(4 * words_per_draw * C), o_bits1 = take(4 * words_per_draw * C);
    const size_t o_ak = take(8 * np * acc_cap), o_am = take(8 * np * acc_cap);
    const size_t o_bk = take(8 * band_total_cap), o_bm = take(8 * band_total_cap), o_bw = take(band_total_cap);
    const size_t o_st = take(sizeof(AcceptState) * np);
    const size_t o_gt = take(sizeof(GenArgs) * np * R), o_ct = take(sizeof(ContractArgs) * np * R);
    const size_t o_rt = take(sizeof(RecheckArgs) * np), o_rta = take(sizeof(RecheckArgs) * np);
    const size_t o_pr = take(sizeof(PoolRec) * np);
    const size_t noff = np + groups.size();   // tile offsets: nprob_g + 1 per group
    const size_t o_off = take(4 * 2 * noff);
    if (off > B.ws_bytes) {
        if (B.exec) hipGraphExecDestroy(B.exec);
        if (B.graph) hipGraphDestroy(B.graph);
        B.exec = nullptr;
        B.graph = nullptr;
        B.sig.clear();
        hipFree(B.ws);
        B.ws = nullptr;
        B.ws_bytes = 0;
        RR_HIP(hipMalloc(&B.ws, off));
        B.ws_bytes = off;
    }
    char* base = (char*)B.ws;
    float* d_hi = (float*)(base + o_hi);
    float* d_lo = (float*)(base + o_lo);
    float* d_m = (float*)(base + o_m);
    uint32_t* d_bits[2] = {(uint32_t*)(base + o_bits0), (uint32_t*)(base + o_bits1)};
    uint64_t* d_ak = (uint64_t*)(base + o_ak);
    double* d_am = (double*)(base + o_am);
    uint64_t* d_bk = (uint64_t*)(base + o_bk);
    double* d_bm = (double*)(base + o_bm);
    uint8_t* d_bw = (uint8_t*)(base + o_bw);
    AcceptState* d_st = (AcceptState*)(base + o_st);
    GenArgs* d_gt = (GenArgs*)(base + o_gt);
    ContractArgs* d_ct = (ContractArgs*)(base + o_ct);
    RecheckArgs* d_rt = (RecheckArgs*)(base + o_rt);
    RecheckArgs* d_rta = (RecheckArgs*)(base + o_rta);
    PoolRec* d_pr = (PoolRec*)(base + o_pr);
    uint32_t* d_off = (uint32_t*)(base + o_off);

    // ---- tables: [round][group order] for generation / contraction; pool order elsewhere
    std::vector<GenArgs> gt(np * R);
    std::vector<ContractArgs> ct(np * R);
    std::vector<RecheckArgs> rt(np), rta(np);
    bool any_refine = false;
    std::vector<PoolRec> pr(np);
    std::vector<size_t> gpos(groups.size());   // first table slot of each group within a round
    {
        size_t pos = 0;
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            gpos[gi] = pos;
            pos += groups[gi].idx.size();
        }
    }
    std::vector<int64_t> rt_order;   // pools in group order (recheck tables per group)
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const Group& g = groups[gi];
        for (size_t j = 0; j < g.idx.size(); ++j) {
            const int64_t i = g.idx[j];
            const Problem& Q = P[i]->P;
            const ContractArgs proto = make_contract_args(Q, precision, bound_constants(Q, precision));
            for (uint64_t r = 0; r < R; ++r) {
                const uint64_t d0 = rbeg[r], cnt = rcnt[r];
                const size_t slot = r * np + gpos[gi] + j;
                uint32_t* bits = d_bits[r & 1] + g.bits_off + j * C * 8 * g.S;
                GenArgs ga{};
                ga.seed = seeds[i];
                ga.key_begin = key_begin + d0;
                ga.num = cnt;
                ga.n = (int)Q.n;
                ga.n1 = (int)Q.n1;
                ga.out = bits;
                gt[slot] = ga;
                ContractArgs ca = proto;
                ca.bits = bits;
                ca.num = cnt;
                ca.key_begin = key_begin + d0;
                ca.out_hi = d_hi + (size_t)i * N + d0;
                ca.out_lo = d_lo + (size_t)i * N + d0;
                ca.out_m32 = d_m + (size_t)i * N + d0;
                ct[slot] = ca;
            }
            RecheckArgs ra{};
            ra.X64 = Q.X64;
            ra.keys = d_bk + boff[i];
            ra.count = &d_st[i].band_count;
            ra.cap = bcap[i];
            ra.seed = seeds[i];
            ra.n = (int)Q.n;
            ra.n1 = (int)Q.n1;
            ra.d = (int)Q.d;
            ra.scale = Q.scale;
            ra.maxmode = Q.metric == RR_METRIC_MAX_SMD ? 1 : 0;
            ra.out = d_bm + boff[i];
            rt[gpos[gi] + j] = ra;
            // small d: the draws accepted outright are recomputed in FP64 as well (cap 0 skips)
            RecheckArgs rf = ra;
            rf.keys = d_ak + (size_t)i * acc_cap;
            rf.count = &d_st[i].acc_count;
            rf.cap = refine_accepted(Q, precision) ? acc_cap : 0u;
            rf.out = d_am + (size_t)i * acc_cap;
            rta[gpos[gi] + j] = rf;
            any_refine = any_refine || refine_accepted(Q, precision);
            rt_order.push_back(i);
        }
    }
    for (int64_t i = 0; i < nprob; ++i) {
        PoolRec q{};
        q.hi = d_hi + (size_t)i * N;
        q.lo = d_lo + (size_t)i * N;
        q.m = d_m + (size_t)i * N;
        q.key_begin = key_begin;
        q.acc_key = d_ak + (size_t)i * acc_cap;
        q.acc_m = d_am + (size_t)i * acc_cap;
        q.acc_cap = acc_cap;
        q.band_key = d_bk + boff[i];
        q.band_m = d_bm + boff[i];
        q.band_work = d_bw + boff[i];
        q.band_cap = bcap[i];
        q.st = d_st + i;
        q.out_key = d_keys[i];
        q.out_m = d_M[i];
        q.capacity = capacity;
        q.a = chi2 ? chi2_quantile_of(q_in, (double)P[i]->P.d) : q_or_a;
        pr[i] = q;
    }
    // tables go up before the graph runs (plain copies, not graph nodes)
    RR_HIP(hipMemcpyAsync(d_gt, gt.data(), sizeof(GenArgs) * gt.size(), hipMemcpyHostToDevice, B.s_main));
    RR_HIP(hipMemcpyAsync(d_ct, ct.data(), sizeof(ContractArgs) * ct.size(), hipMemcpyHostToDevice, B.s_main));
    RR_HIP(hipMemcpyAsync(d_rt, rt.data(), sizeof(RecheckArgs) * rt.size(), hipMemcpyHostToDevice, B.s_main));
    RR_HIP(hipMemcpyAsync(d_rta, rta.data(), sizeof(RecheckArgs) * rta.size(), hipMemcpyHostToDevice, B.s_main));
    RR_HIP(hipMemcpyAsync(d_pr, pr.data(), sizeof(PoolRec) * pr.size(), hipMemcpyHostToDevice, B.s_main));
    RR_HIP(hipStreamSynchronize(B.s_main));

    // ---- graph: captured once per distinct argument set (tiles included), then launched,
    // ordered after the caller's stream and before its later work; returns the graph's GPU time
    auto launch_graph = [&](float* out_ms) -> rr_status {
        std::vector<uint64_t> sig;
        sig.push_back((uint64_t)nprob);
        sig.push_back(key_begin);
        sig.push_back(N);
        sig.push_back((uint64_t)mode | (chi2 ? 0x100u : 0u));
        uint64_t qbits;
        std::memcpy(&qbits, &q_or_a, 8);
        sig.push_back(qbits);
        sig.push_back((uint64_t)precision);
        sig.push_back(capacity);
        sig.push_back((uint64_t)(uintptr_t)B.ws);
        sig.push_back(C);
        for (int64_t i = 0; i < nprob; ++i) {
            // the handle's process-unique id, not its address: a freed handle's address can be
            // reused by a new problem of another shape, whose S group, tile grid and operands the
            // captured launches would not match
            sig.push_back(P[i]->P.uid);
            sig.push_back(seeds[i]);
            sig.push_back((uint64_t)(uintptr_t)d_keys[i]);
            sig.push_back((uint64_t)(uintptr_t)d_M[i]);
        }
        for (const Group& g : groups) sig.push_back(((uint64_t)g.tune.db << 32) | (uint32_t)g.tune.gen_wg);
        if (!B.exec || sig != B.sig) {
            if (B.exec) hipGraphExecDestroy(B.exec);
            if (B.graph) hipGraphDestroy(B.graph);
            B.exec = nullptr;
            B.graph = nullptr;
            B.sig.clear();
            // Every capture starts from streams and events that have never been captured, so
            // that none carries capture state (the nodes its last record or wait referred to)
            // from a graph that has been destroyed; the timing and ordering events recorded
            // outside the graph go with the old streams too, so that no event is re-recorded
            // after its stream is gone.  Nothing runs on the old ones now: the last launch was
            // synchronised, and so were the tables' copies.
            for (hipEvent_t ev : B.ev) hipEventDestroy(ev);
            B.ev.clear();
            for (hipEvent_t* ev : {&B.t0, &B.t1, &B.join}) {
                if (*ev) hipEventDestroy(*ev);
                *ev = nullptr;
            }
            const hipError_t d1 = hipStreamDestroy(B.s_main), d2 = hipStreamDestroy(B.s_gen);
            B.s_main = B.s_gen = nullptr;
            RR_HIP(d1);
            RR_HIP(d2);
            RR_HIP(hipStreamCreateWithFlags(&B.s_main, hipStreamNonBlocking));
            RR_HIP(hipStreamCreateWithFlags(&B.s_gen, hipStreamNonBlocking));
            RR_HIP(hipEventCreate(&B.t0));
            RR_HIP(hipEventCreate(&B.t1));
            RR_HIP(hipEventCreateWithFlags(&B.join, hipEventDisableTiming));
            const size_t nev = 2 * R * groups.size() + 4;
            while (B.ev.size() < nev) {
                hipEvent_t e;
                RR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
                B.ev.push_back(e);
            }
            hipEvent_t* ready = B.ev.data();                          // [r][group]
            hipEvent_t* freed = B.ev.data() + R * groups.size();      // [r][group]
            hipEvent_t fork = B.ev[2 * R * groups.size()], join = B.ev[2 * R * groups.size() + 1];
            hipEvent_t fork2 = B.ev[2 * R * groups.size() + 2], join2 = B.ev[2 * R * groups.size() + 3];
            int64_t kernels = 0;
            hipError_t e = hipStreamBeginCapture(B.s_main, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) {
                set_error(std::string("rr_draw_balance_batched: graph capture: ") + hipGetErrorString(e));
                return RR_E_DEVICE;
            }
            auto check = [&](hipError_t x) {
                if (e == hipSuccess) e = x;
            };
            hipLaunchKernelGGL(batch_init_kernel, dim3((unsigned)((nprob + 255) / 256)), dim3(256), 0, B.s_main, d_st,
                               (int)nprob, (uint32_t)k);
            check(hipGetLastError());
            ++kernels;
            check(hipEventRecord(fork, B.s_main));
            check(hipStreamWaitEvent(B.s_gen, fork, 0));
            for (uint64_t r = 0; r < R && e == hipSuccess; ++r) {
                const uint64_t cnt = rcnt[r];
                for (size_t gi = 0; gi < groups.size(); ++gi) {
                    const Group& g = groups[gi];
                    const uint64_t m = g.idx.size();
                    if (r >= 2) check(hipStreamWaitEvent(B.s_gen, freed[(r - 2) * groups.size() + gi], 0));
                    const uint64_t gen_wgs = std::min<uint64_t>((m * cnt + 3) / 4, (uint64_t)cus * g.tune.gen_wg);
                    check(launch_gen_batch(g.S, d_gt + r * np + gpos[gi], m, cnt, (int)gen_wgs, B.s_gen));
                    check(hipEventRecord(ready[r * groups.size() + gi], B.s_gen));
                    check(hipStreamWaitEvent(B.s_main, ready[r * groups.size() + gi], 0));
                    ContractArgs a0{};
                    a0.tab = d_ct + r * np + gpos[gi];
                    a0.tpp = (uint32_t)((cnt + g.tile - 1) / g.tile);
                    a0.nprob = (uint32_t)m;
                    const uint64_t tiles = m * a0.tpp;
                    check(launch_contract(g.S, precision, g.tune.db, true, a0, (int)std::min<uint64_t>(tiles, cus),
                                          B.s_main));
                    check(hipEventRecord(freed[r * groups.size() + gi], B.s_main));
                    kernels += 2;
                }
            }
            check(hipEventRecord(join, B.s_gen));
            check(hipStreamWaitEvent(B.s_main, join, 0));
            hipLaunchKernelGGL(batch_select_kernel, dim3((unsigned)nprob), dim3(1024), 0, B.s_main, d_pr, (uint32_t)N,
                               mode);
            check(hipGetLastError());
            ++kernels;
            // the groups' rechecks are independent: alternate them over the two streams
            check(hipEventRecord(fork2, B.s_main));
            check(hipStreamWaitEvent(B.s_gen, fork2, 0));
            for (size_t gi = 0; gi < groups.size(); ++gi) {
                const int rgrid = kBatchRecheckWgsPerCu * cus;
                check(launch_recheck_batch(groups[gi].S, d_rt + gpos[gi], (int)groups[gi].idx.size(),
                                           d_off + gpos[gi] + gi, rgrid, (gi & 1) ? B.s_gen : B.s_main));
                kernels += 2;
                if (any_refine) {
                    check(launch_recheck_batch(groups[gi].S, d_rta + gpos[gi], (int)groups[gi].idx.size(),
                                               d_off + noff + gpos[gi] + gi, rgrid, (gi & 1) ? B.s_gen : B.s_main));
                    kernels += 2;
                }
            }
            check(hipEventRecord(join2, B.s_gen));
            check(hipStreamWaitEvent(B.s_main, join2, 0));
            hipLaunchKernelGGL(batch_finish_kernel, dim3((unsigned)nprob), dim3(1024), 0, B.s_main, d_pr, mode);
            check(hipGetLastError());
            ++kernels;
            hipGraph_t graph = nullptr;
            const hipError_t e2 = hipStreamEndCapture(B.s_main, &graph);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&B.exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                if (graph) hipGraphDestroy(graph);
                B.exec = nullptr;
                set_error(std::string("rr_draw_balance_batched: graph build: ") + hipGetErrorString(e));
                return RR_E_DEVICE;
            }
            B.graph = graph;
            B.sig = sig;
            B.kernels = kernels;
        }

        RR_HIP(hipEventRecord(B.join, st));
        RR_HIP(hipStreamWaitEvent(B.s_main, B.join, 0));
        RR_HIP(hipEventRecord(B.t0, B.s_main));
        RR_HIP(hipGraphLaunch(B.exec, B.s_main));
        RR_HIP(hipEventRecord(B.t1, B.s_main));
        RR_HIP(hipStreamSynchronize(B.s_main));
        RR_HIP(hipEventElapsedTime(out_ms, B.t0, B.t1));
        return RR_OK;
    };

    // ---- per-class tiles: the choice of each bitmask class read from the tune file, else the
    // defaults above.  Candidates are not measured inside the graph here: a version that
    // recaptured the whole graph once per candidate ended in a host segmentation fault of
    // unknown cause, so that path is switched off.
    float graph_ms = 0.f;
    {
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            Tune t{};
            if (batch_tune_lookup(precision, groups[gi].S, &t)) {
                groups[gi].tune = t;
                groups[gi].tile = contract_tile(precision, groups[gi].S, t.db);
            }
        }
        const rr_status ls = launch_graph(&graph_ms);
        if (ls != RR_OK) return ls;
    }
    std::vector<AcceptState> hs(np);
    RR_HIP(hipMemcpy(hs.data(), d_st, sizeof(AcceptState) * np, hipMemcpyDeviceToHost));
    uint64_t band_total = 0;
    rr_status result = RR_OK;
    uint64_t* sk[2] = {nullptr, nullptr};
    uint32_t* si[2] = {nullptr, nullptr};
    for (int64_t i = 0; i < nprob && result == RR_OK; ++i) {
        const AcceptState& a = hs[i];
        band_total += a.band_count;
        if (a.overflow || a.guard_fail) {
            // guard band beyond the batched capacity: the single-pool pipeline decides this pool,
            // on the caller's stream (ordered after the graph, which has completed), so that the
            // pool's handle records its events only on streams that outlive this batch's own
            const double keep_ms = graph_ms;
            RR_HIP(hipEventRecord(B.join, B.s_main));
            RR_HIP(hipStreamWaitEvent(st, B.join, 0));
            rr_status s = draw_pipeline(P[i]->P, false, seeds[i], key_begin, N, chi2 ? RR_MODE_CHI2_QUANTILE : mode,
                                        chi2 ? q_in : q_or_a, precision, d_keys[i], d_M[i], nullptr, capacity,
                                        &h_counts[i], st, nullptr);
            graph_ms = keep_ms;
            if (s != RR_OK) result = s;
            continue;
        }
        const uint64_t K = a.acc_count;
        h_counts[i] = K;
        if (K > capacity) {
            set_error("rr_draw_balance_batched: capacity below the accepted count");
            result = RR_E_CAPACITY;
            break;
        }
        if (mode == RR_MODE_QUANTILE && K != k) {
            set_error("rr_draw_balance_batched: accepted count differs from k");
            result = RR_E_DEVICE;
            break;
        }
        if (!a.done && K > 0) {
            // more accepted keys than one workgroup sorts in LDS
            if (!sk[0]) {
                size_t bytes = 0;
                for (int64_t j = 0; j < nprob; ++j) bytes = std::max<size_t>(bytes, hs[j].acc_count);
                hipError_t x = hipSuccess;
                for (int t = 0; t < 2 && x == hipSuccess; ++t) {
                    x = hipMalloc(&sk[t], 8 * bytes);
                    if (x == hipSuccess) x = hipMalloc(&si[t], 4 * bytes);
                }
                if (x != hipSuccess) {
                    set_error(std::string("rr_draw_balance_batched: ") + hipGetErrorString(x));
                    result = RR_E_DEVICE;
                    break;
                }
            }
            hipError_t x = sort_accepted(pr[i].acc_key, pr[i].acc_m, nullptr, (uint32_t)K, sk, si, d_keys[i], d_M[i],
                                         nullptr, B.s_main);
            if (x == hipSuccess) x = hipStreamSynchronize(B.s_main);
            if (x != hipSuccess) {
                set_error(std::string("rr_draw_balance_batched: ") + hipGetErrorString(x));
                result = RR_E_DEVICE;
            }
        }
    }
    for (int t = 0; t < 2; ++t) {
        hipFree(sk[t]);
        hipFree(si[t]);
    }
    if (result != RR_OK) return result;
    RR_HIP(hipEventRecord(B.join, B.s_main));
    RR_HIP(hipStreamWaitEvent(st, B.join, 0));
    const double total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    set_timing(total, graph_ms, 0.0, B.kernels, band_total);
    return RR_OK;
}
