// Host-logic checks of librr against the mock runtime (tests/hostmock/mock_hip.cpp), built with
// AddressSanitizer / UBSan.  Kernels do not run, so every device result reads as zero (or, with
// RR_MOCK_FLAGS_SET, the batched per-pool states as all flags set); the checks are about the
// host code: its memory safety, the lifetimes of its streams / events / graphs, when a batched
// call captures a new graph, workspace reuse across handles, and that the allocation-free entry
// point allocates nothing.
//
// Usage: driver SHAPES_FILE (lines "n n1 d": the pools of the 512-pool batched workload).
// Prints "CHECK <name> ok" per check and "ALL OK" at the end; exits 1 on the first failure.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include <hip/hip_runtime.h>

#include "rr.h"

extern "C" long mock_violations();
extern "C" long mock_captures();
extern "C" long mock_mallocs();
extern "C" long mock_frees();

namespace {

void check(bool ok, const char* name) {
    if (!ok || mock_violations()) {
        std::printf("CHECK %s FAILED (mock violations %ld; last error: %s)\n", name, mock_violations(),
                    rr_last_error());
        std::exit(1);
    }
    std::printf("CHECK %s ok\n", name);
}

struct Pool {
    rr_problem* P = nullptr;
    void* X = nullptr;
};

Pool prep(int n, int n1, int d, double ridge = 1e-2) {
    Pool p;
    hipMalloc(&p.X, sizeof(float) * (size_t)n * d);
    float* x = static_cast<float*>(p.X);
    for (long i = 0; i < (long)n * d; ++i) x[i] = (float)((i * 2654435761u) % 1000) / 1000.0f;
    const rr_status s = rr_prepare(p.X, RR_X_FP32, n, d, d, n1, ridge, nullptr, &p.P);
    if (s != RR_OK) {
        std::printf("prepare n=%d d=%d failed: %s\n", n, d, rr_last_error());
        std::exit(1);
    }
    return p;
}

void release(Pool& p) {
    rr_free(p.P);
    hipFree(p.X);
    p = Pool{};
}

// Outputs of one batched call (allocated before the call, so that allocation counts around the
// call see only the library's own).
struct Outs {
    std::vector<void*> keys, M;
    std::vector<uint64_t> counts;
    Outs(size_t np, uint64_t cap) : counts(np, 0) {
        for (size_t i = 0; i < np; ++i) {
            void *k, *m;
            hipMalloc(&k, 8 * (cap ? cap : 1));
            hipMalloc(&m, 8 * (cap ? cap : 1));
            keys.push_back(k);
            M.push_back(m);
        }
    }
    ~Outs() {
        for (void* p : keys) hipFree(p);
        for (void* p : M) hipFree(p);
    }
};

// A batched call into `o` (the captured graph is keyed on the output pointers too: the same
// outputs are needed for a replay).
rr_status batched_into(Outs& o, std::vector<Pool>& ps, uint64_t seed0, uint64_t key_begin, uint64_t N, int mode,
                       double qa, int prec, uint64_t cap, long* captures = nullptr) {
    std::vector<rr_problem*> H;
    std::vector<uint64_t> seeds;
    for (size_t i = 0; i < ps.size(); ++i) {
        H.push_back(ps[i].P);
        seeds.push_back(seed0 + i);
    }
    const long c0 = mock_captures();
    const rr_status s = rr_draw_balance_batched(H.data(), (int64_t)H.size(), seeds.data(), key_begin, N, mode, qa,
                                                prec, reinterpret_cast<uint64_t* const*>(o.keys.data()),
                                                reinterpret_cast<double* const*>(o.M.data()), cap, o.counts.data(),
                                                nullptr);
    if (captures) *captures = mock_captures() - c0;
    return s;
}

rr_status batched(std::vector<Pool>& ps, uint64_t seed0, uint64_t key_begin, uint64_t N, int mode, double qa,
                  int prec, uint64_t cap, long* captures = nullptr) {
    Outs o(ps.size(), cap);
    return batched_into(o, ps, seed0, key_begin, N, mode, qa, prec, cap, captures);
}

rr_status single(Pool& p, uint64_t seed, uint64_t N, int mode, double qa, int prec, uint64_t cap,
                 long* mallocs = nullptr) {
    void *k, *m, *f;
    hipMalloc(&k, 8 * cap);
    hipMalloc(&m, 8 * cap);
    hipMalloc(&f, cap);
    uint64_t cnt = 0;
    const long a0 = mock_mallocs();
    const rr_status s = rr_draw_balance(p.P, seed, 0, N, mode, qa, prec, static_cast<uint64_t*>(k),
                                        static_cast<double*>(m), static_cast<uint8_t*>(f), cap, &cnt, nullptr);
    if (mallocs) *mallocs = mock_mallocs() - a0;
    hipFree(k);
    hipFree(m);
    hipFree(f);
    return s;
}

}  // namespace

int main(int argc, char** argv) {
    std::vector<int> shapes;   // n, n1, d triples
    if (argc > 1) {
        FILE* f = std::fopen(argv[1], "r");
        int n, n1, d;
        while (f && std::fscanf(f, "%d %d %d", &n, &n1, &d) == 3) {
            shapes.push_back(n);
            shapes.push_back(n1);
            shapes.push_back(d);
        }
        if (f) std::fclose(f);
    }
    const int T = RR_MODE_THRESHOLD;   // threshold mode: zero device results are a valid outcome
    const int precs[4] = {RR_PREC_SPLIT_BF16, RR_PREC_FP32, RR_PREC_FIXED_I8, RR_PREC_GRAM_BF16};
    const int sh12[12][2] = {{50, 10}, {61, 3}, {200, 40}, {300, 33}, {257, 100}, {700, 64}, {1000, 250},
                             {1024, 500}, {1500, 130}, {2000, 500}, {2000, 500}, {99, 98}};

    // Batched calls over every bitmask class and operand form, and single-pool calls on the
    // same handles; the pools are released at the end of each block.
    for (int prec : precs) {
        std::vector<Pool> ps;
        for (auto& s : sh12) ps.push_back(prep(s[0], s[0] / 2, s[1]));
        long cap1 = 0, cap2 = 0;
        Outs o(ps.size(), 3000);
        const rr_status s1 = batched_into(o, ps, 900, 0, 3000, T, 50.0, prec, 3000, &cap1);
        const rr_status s2 = batched_into(o, ps, 900, 0, 3000, T, 50.0, prec, 3000, &cap2);
        check(s1 == RR_OK && s2 == RR_OK, "batched call, every bitmask class");
        check(cap1 == 1 && cap2 == 0, "graph captured once, replayed for the same arguments");
        for (auto& p : ps) check(single(p, 900, 3000, T, 50.0, prec, 3000) == RR_OK, "single-pool call on the handles");
        for (auto& p : ps) release(p);
    }
    {
        std::vector<Pool> ps;
        ps.push_back(prep(120, 60, 12));
        ps.push_back(prep(640, 320, 64));
        long c = 0;
        Outs o(ps.size(), 30000);
        check(batched_into(o, ps, 970, 0, 30000, T, 40.0, RR_PREC_SPLIT_BF16, 30000, &c) == RR_OK && c == 1,
              "first call");
        check(batched_into(o, ps, 987, 5, 30000, T, 40.0, RR_PREC_SPLIT_BF16, 30000, &c) == RR_OK && c == 1,
              "new seeds and key range: a new graph");
        // one pool's handle replaced by a problem of another shape (and bitmask class)
        release(ps[1]);
        ps[1] = prep(1500, 750, 70);
        check(batched_into(o, ps, 987, 5, 30000, T, 40.0, RR_PREC_SPLIT_BF16, 30000, &c) == RR_OK && c == 1,
              "replaced handle with the same arguments: a new graph");
        check(batched_into(o, ps, 987, 5, 30000, T, 40.0, RR_PREC_SPLIT_BF16, 30000, &c) == RR_OK && c == 0,
              "then replayed");
        Outs o2(ps.size(), 30000);
        check(batched_into(o2, ps, 987, 5, 30000, T, 40.0, RR_PREC_SPLIT_BF16, 30000, &c) == RR_OK && c == 1,
              "new output buffers: a new graph");
        for (auto& p : ps) release(p);
    }
    {
        // argument errors and capacity, with the pools kept alive into the next block and
        // released in its middle
        std::vector<Pool> errs;
        errs.push_back(prep(60, 30, 5));
        errs.push_back(prep(80, 40, 6));
        check(batched(errs, 990, 0, 1000, RR_MODE_QUANTILE, 0.1, RR_PREC_SPLIT_BF16, 50) == RR_E_CAPACITY,
              "capacity below q N");
        check(batched(errs, 990, 0, 1000, RR_MODE_QUANTILE, 1.5, RR_PREC_SPLIT_BF16, 1000) == RR_E_ARG, "q > 1");
        batched(errs, 990, 0, 1000, T, 1e9, RR_PREC_SPLIT_BF16, 10);
        check(true, "threshold above every draw with a small capacity");
        std::vector<Pool> ps;
        const size_t np = shapes.size() / 3;
        for (size_t p = 0; p < np; ++p) {
            ps.push_back(prep(shapes[3 * p], shapes[3 * p + 1], shapes[3 * p + 2]));
            if (p == np / 2)
                for (auto& e : errs) release(e);
        }
        if (np) {
            check(batched(ps, 1592591616, 0, 100000, T, 30.0, RR_PREC_SPLIT_BF16, 100000) == RR_OK,
                  "the 512-pool workload");
            for (size_t i = 0; i < np; i += np / 8) single(ps[i], 77, 100000, T, 30.0, RR_PREC_SPLIT_BF16, 100000);
        }
        for (auto& p : ps) release(p);
    }
    {
        // a released handle's workspaces go to the next handle on the device: its first call
        // allocates nothing
        Pool a = prep(300, 150, 40);
        check(single(a, 5, 200000, T, 20.0, RR_PREC_SPLIT_BF16, 200000) == RR_OK, "call on a first handle");
        release(a);
        Pool b = prep(300, 150, 40);
        long m = -1;
        check(single(b, 5, 200000, T, 20.0, RR_PREC_SPLIT_BF16, 200000, &m) == RR_OK && m == 0,
              "the next handle's first call reuses the released workspace");
        release(b);
    }
    {
        // the allocation-free entry point: no allocation or free, on two calls in a row
        Pool p = prep(300, 120, 40);
        void *keys, *m32, *err, *m64;
        hipMalloc(&keys, 8 * 4096);
        hipMalloc(&m32, 4 * 4096);
        hipMalloc(&err, 4 * 4096);
        hipMalloc(&m64, 8 * 4096);
        const long a0 = mock_mallocs(), f0 = mock_frees();
        const rr_status s1 = rr_balance_keys_noalloc(p.P, 3, 0, static_cast<const uint64_t*>(keys), 4096,
                                                     RR_PREC_SPLIT_BF16, static_cast<float*>(m32),
                                                     static_cast<float*>(err), static_cast<double*>(m64), nullptr);
        const rr_status s2 = rr_balance_keys_noalloc(p.P, 3, 0, static_cast<const uint64_t*>(keys), 1000,
                                                     RR_PREC_FIXED_I8, static_cast<float*>(m32),
                                                     static_cast<float*>(err), static_cast<double*>(m64), nullptr);
        check(s1 == RR_OK && s2 == RR_OK && mock_mallocs() == a0 && mock_frees() == f0,
              "allocation-free entry point allocates and frees nothing");
        void *k, *M, *fl, *cnt, *st;
        hipMalloc(&k, 8 * 4096);
        hipMalloc(&M, 8 * 4096);
        hipMalloc(&fl, 4096);
        hipMalloc(&cnt, 8);
        hipMalloc(&st, 4);
        check(rr_draw_balance_async(p.P, 3, 0, 100000, T, 10.0, RR_PREC_SPLIT_BF16, static_cast<uint64_t*>(k),
                                    static_cast<double*>(M), static_cast<uint8_t*>(fl), 4096,
                                    static_cast<uint64_t*>(cnt), static_cast<int32_t*>(st), nullptr) == RR_OK,
              "stream-ordered call");
        for (void* q : {keys, m32, err, m64, k, M, fl, cnt, st}) hipFree(q);
        release(p);
    }
    {
        // one handle used from several caller streams in turn, one of them destroyed between
        // calls: the handle's events must never be re-recorded after their stream is gone
        Pool p = prep(200, 100, 20);
        hipStream_t a, b, c;
        hipStreamCreateWithFlags(&a, hipStreamNonBlocking);
        hipStreamCreateWithFlags(&b, hipStreamNonBlocking);
        void *k, *M, *fl, *cnt, *st;
        hipMalloc(&k, 8 * 60000);
        hipMalloc(&M, 8 * 60000);
        hipMalloc(&fl, 60000);
        hipMalloc(&cnt, 8);
        hipMalloc(&st, 4);
        uint64_t hc = 0;
        auto on = [&](hipStream_t s, bool async) {
            return async ? rr_draw_balance_async(p.P, 9, 0, 60000, T, 5.0, RR_PREC_SPLIT_BF16,
                                                 static_cast<uint64_t*>(k), static_cast<double*>(M),
                                                 static_cast<uint8_t*>(fl), 60000, static_cast<uint64_t*>(cnt),
                                                 static_cast<int32_t*>(st), s)
                         : rr_draw_balance(p.P, 9, 0, 60000, T, 5.0, RR_PREC_SPLIT_BF16, static_cast<uint64_t*>(k),
                                           static_cast<double*>(M), static_cast<uint8_t*>(fl), 60000, &hc, s);
        };
        check(on(a, true) == RR_OK && on(a, false) == RR_OK, "calls on a first stream");
        check(on(b, false) == RR_OK, "then on a second stream");
        hipStreamDestroy(a);
        hipStreamCreateWithFlags(&c, hipStreamNonBlocking);
        check(on(c, true) == RR_OK && on(b, false) == RR_OK && on(nullptr, false) == RR_OK,
              "after the first stream is destroyed: a third stream, the second, the null stream");
        hipStreamDestroy(b);
        hipStreamDestroy(c);
        for (void* q : {k, M, fl, cnt, st}) hipFree(q);
        release(p);
        check(true, "handle released after its streams were destroyed");
    }
    {
        // tuning-size calls: the autotuner probes on the calling handle before the call runs
        Pool p = prep(1100, 550, 17, 0.0);
        check(single(p, 91, 1u << 20, T, 10.0, RR_PREC_FIXED_I8, 1u << 20) == RR_OK, "first call of a tuning bucket");
        check(single(p, 91, 1u << 23, T, 10.0, RR_PREC_SPLIT_BF16, 1u << 20) == RR_OK, "chunk-length tuning call");
        release(p);
    }
    check(mock_violations() == 0, "no runtime-rule violations");
    std::printf("ALL OK\n");
    return 0;
}
