// Autotuner of the draw pipeline's launch configuration.
//
// Tunables: the contraction tile (db = 32-draw blocks per wave, 1 or 2, where the tile's
// bitmasks fit in LDS) and the generation kernel's workgroups per CU (2 up to the number that
// fits beside one contraction workgroup by registers, at most 4).  Neither changes any
// result: per-draw arithmetic depends only on the covariate chunking, which is fixed.
//
// Buckets: (precision, S = 256-unit chunks per draw, floor(log2(ks * ncb))), i.e. the
// bitmask length and the MFMA work per draw.  On the first Monte Carlo call of a bucket that
// covers at least 2^20 draws, every candidate runs the full two-stream pipeline on the calling
// problem for a probe pool of 2^18 .. 2^20 draws (about 2^42 MFMA flops, so several chunks
// overlap as in a long call), timed on the host around the synchronised call (best of two
// after a warm-up run); the fastest wins.  Results live for the
// process; with RR_TUNE_FILE set they are also read from and appended to that JSON file.
// RR_TUNE=0 disables probing (defaults everywhere).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "rr_internal.h"

namespace rr {

// Generation workgroups (4 waves, one per SIMD) that fit on a CU beside one contraction
// workgroup, by vector registers: a SIMD holds 512 per lane, allocated in steps of 8.  If the
// generation kernel takes more, the contraction workgroup cannot start on that CU until the
// persistent generation grid has drained, and the two kernels no longer overlap.
int gen_wg_fit(int prec, int S, int db, bool batch) {
    auto r8 = [](int v) { return (v + 7) & ~7; };
    const int c = contract_kernel_vgprs(prec, S, db, batch), g = gen_kernel_vgprs(S, batch);
    if (c <= 0 || g <= 0) return kGenWgPerCu;
    const int free_regs = 512 - (contract_waves(prec, S) / 4) * r8(c);
    return std::max(1, std::min(4, free_regs / r8(g)));
}

Tune tune_default(int prec, int S, bool batch) {
    const int db = contract_db_default(prec, S);
    return Tune{db, std::min(kGenWgPerCu, gen_wg_fit(prec, S, db, batch))};
}

namespace {

using Key = std::tuple<int, int, int>;   // precision, S, floor(log2(ks * ncb))

struct Entry {
    Tune t;
    double ms;
};

std::mutex g_mu;
std::map<Key, Entry> g_cache;
bool g_loaded = false;

int cost_log2(const Problem& P, int prec) {
    uint64_t c = (uint64_t)P.ks * (uint64_t)(prec == RR_PREC_GRAM_BF16 ? P.ncb_gram : P.ncb);
    int l = 0;
    while (c > 1) {
        c >>= 1;
        ++l;
    }
    return l;
}

const char* tune_file() {
    const char* f = std::getenv("RR_TUNE_FILE");
    return (f && *f) ? f : nullptr;
}

bool tuning_enabled() {
    const char* e = std::getenv("RR_TUNE");
    return !(e && std::strcmp(e, "0") == 0);
}

// One entry per line: {"prec": P, "S": S, "cost_log2": C, "db": D, "gen_wg": G, "ms": T}
void load_file() {
    g_loaded = true;
    const char* path = tune_file();
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        const char* p = std::strchr(line, '{');
        if (!p) continue;
        int prec, S, cl, db, gw;
        double ms;
        if (std::sscanf(p, "{\"prec\": %d, \"S\": %d, \"cost_log2\": %d, \"db\": %d, \"gen_wg\": %d, \"ms\": %lf",
                        &prec, &S, &cl, &db, &gw, &ms) == 6 &&
            contract_db_ok(prec, S, db) && gw >= 1 && gw <= 8)
            g_cache[Key(prec, S, cl)] = Entry{Tune{db, gw}, ms};
    }
    std::fclose(f);
}

void save_file() {
    const char* path = tune_file();
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\"rr_tune\": [\n");
    size_t i = 0;
    for (const auto& kv : g_cache) {
        std::fprintf(f, "  {\"prec\": %d, \"S\": %d, \"cost_log2\": %d, \"db\": %d, \"gen_wg\": %d, \"ms\": %.4f}%s\n",
                     std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), kv.second.t.db,
                     kv.second.t.gen_wg, kv.second.ms, ++i < g_cache.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

}  // namespace

Tune tune_for(Problem& P, int prec, bool exact, uint64_t work_draws, hipStream_t st, bool probe) {
    const Tune def = tune_default(prec, P.S, false);
    if (exact || !tuning_enabled()) return def;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_loaded) load_file();
    const Key key(prec, P.S, cost_log2(P, prec));
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        // entries read from a file may come from another build: keep them within the fit
        Tune t = it->second.t;
        t.gen_wg = std::min(t.gen_wg, gen_wg_fit(prec, P.S, t.db, false));
        return t;
    }
    if (work_draws < (1u << 20) || !probe) return def;

    // probe pool: ~2^42 MFMA flops, 2^18 .. 2^20 draws
    const double ncb = (double)(prec == RR_PREC_GRAM_BF16 ? P.ncb_gram : P.ncb);
    const double flops_per_draw =
        2.0 * 16.0 * (double)P.ks * 32.0 * ncb * (prec == RR_PREC_SPLIT_BF16 || prec == RR_PREC_GRAM_BF16 ? 2.0 : 1.0);
    uint64_t N = (uint64_t)(std::ldexp(1.0, 42) / std::max(1.0, flops_per_draw));
    N = std::min<uint64_t>(std::max<uint64_t>(N, 1u << 18), 1u << 20);
    const double q = 1e-3;
    const uint64_t cap = (uint64_t)std::ceil(q * (double)N) + 1;
    uint64_t* keys = nullptr;
    double* M = nullptr;
    if (hipMalloc(&keys, sizeof(uint64_t) * cap) != hipSuccess || hipMalloc(&M, sizeof(double) * cap) != hipSuccess) {
        hipFree(keys);
        return def;
    }
    Tune best = def;
    double best_ms = INFINITY;
    for (int db = 1; db <= 2; ++db) {
        if (!contract_db_ok(prec, P.S, db)) continue;
        const int fit = gen_wg_fit(prec, P.S, db, false);
        for (int gw = std::min(2, fit); gw <= fit; ++gw) {
            const Tune t{db, gw};
            double ms = INFINITY;
            for (int rep = 0; rep < 3; ++rep) {
                uint64_t cnt = 0;
                const auto t0 = std::chrono::steady_clock::now();
                const rr_status s = draw_pipeline(P, false, 0x7u, 0, N, RR_MODE_QUANTILE, q, prec, keys, M, nullptr,
                                                  cap, &cnt, st, &t);
                const double dt =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                if (s != RR_OK) {
                    ms = INFINITY;
                    break;
                }
                if (rep > 0) ms = std::min(ms, dt);   // the first run warms caches and code
            }
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    }
    hipFree(keys);
    hipFree(M);
    if (!std::isfinite(best_ms)) return def;
    g_cache[key] = Entry{best, best_ms};
    save_file();
    return best;
}

}  // namespace rr
