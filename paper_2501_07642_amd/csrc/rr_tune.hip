// Autotuner of the draw pipeline's launch configuration.
//
// Tunables (none changes any result: per-draw arithmetic depends only on the covariate
// chunking, which is fixed, and the acceptance is exact):
//   db        the contraction tile, 32-draw blocks per wave (1 or 2, where the tile's bitmasks
//             fit in LDS beside the operand stages);
//   gen_wg    generation workgroups per CU, from 2 up to the number that fits beside one
//             contraction workgroup by registers (at most 4);
//   chunk     draws per pipeline chunk of a single-pool call, 2^19 .. 2^21 (longer chunks mean
//             fewer launches and events; the first chunk's generation and the last chunk's
//             contraction run without a partner, so shorter chunks waste less at the ends).
// The waves per workgroup, covariate blocks per chunk and LDS stage depth are fixed by the
// register and LDS budget (two 8-wave contraction workgroups' worth of waves per CU beside
// three generation waves per SIMD) rather than tuned.
//
// Single-pool buckets: (precision, S = 256-unit chunks per draw, floor(log2(ks * ncb))), i.e.
// the bitmask length and the MFMA work per draw.  On the first Monte Carlo call of a bucket
// that covers at least 2^20 draws, every (db, gen_wg) candidate runs the full two-stream
// pipeline on the calling problem for a probe pool of 2^18 .. 2^20 draws (about 2^42 MFMA
// flops), timed on the host around the synchronised call (best of two after a warm-up run);
// then, for calls of at least 2^23 draws, the chunk length is chosen the same way on a 2^23-draw
// pool with the winning tile.  Batched launches: per bitmask class (precision, S), a (db,
// gen_wg) choice is taken from the tune file when it holds one ("batched": 1), else the
// defaults; batched calls measure nothing themselves.  Results live for the process; with
// RR_TUNE_FILE set they are also read from and appended to that JSON file, and rr_tune_report
// returns them.  RR_TUNE=0 disables probing (defaults everywhere).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
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

using Key = std::tuple<int, int, int, int>;   // batched, precision, S, floor(log2(ks * ncb)) (-1 batched)

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

// One entry per line: {"batched": B, "prec": P, "S": S, "cost_log2": C, "db": D, "gen_wg": G,
// "chunk_log2": L, "ms": T} ("batched" and "chunk_log2" may be missing: 0 and 20).
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
        int batched = 0, prec, S, cl, db, gw, clog = 20;
        double ms;
        const char* q = std::strstr(p, "\"prec\"");
        if (!q) continue;
        if (const char* b = std::strstr(p, "\"batched\": ")) batched = std::atoi(b + 12);
        if (const char* c = std::strstr(p, "\"chunk_log2\": ")) clog = std::atoi(c + 14);
        const char* m = std::strstr(p, "\"ms\": ");
        if (!m || std::sscanf(m, "\"ms\": %lf", &ms) != 1) continue;
        if (std::sscanf(q, "\"prec\": %d, \"S\": %d, \"cost_log2\": %d, \"db\": %d, \"gen_wg\": %d", &prec, &S, &cl,
                        &db, &gw) == 5 &&
            contract_db_ok(prec, S, db) && gw >= 1 && gw <= 8 && clog >= 16 && clog <= 21) {
            Tune t{db, gw};
            t.chunk_log2 = clog;
            g_cache[Key(batched ? 1 : 0, prec, S, cl)] = Entry{t, ms};
        }
    }
    std::fclose(f);
}

std::string report_json() {
    std::string out = "{\"rr_tune\": [\n";
    size_t i = 0;
    for (const auto& kv : g_cache) {
        char buf[256];
        std::snprintf(buf, sizeof buf,
                      "  {\"batched\": %d, \"prec\": %d, \"S\": %d, \"cost_log2\": %d, \"db\": %d, \"gen_wg\": %d, "
                      "\"chunk_log2\": %d, \"ms\": %.4f}%s\n",
                      std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
                      kv.second.t.db, kv.second.t.gen_wg, kv.second.t.chunk_log2, kv.second.ms,
                      ++i < g_cache.size() ? "," : "");
        out += buf;
    }
    out += "]}\n";
    return out;
}

void save_file() {
    const char* path = tune_file();
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    const std::string doc = report_json();
    std::fputs(doc.c_str(), f);
    std::fclose(f);
    std::rename(tmp.c_str(), path);
}

}  // namespace

Tune tune_for(Problem& P, int prec, bool exact, uint64_t work_draws, hipStream_t st, bool probe) {
    const Tune def = tune_default(prec, P.S, false);
    if (exact || !tuning_enabled()) return def;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_loaded) load_file();
    const Key key(0, prec, P.S, cost_log2(P, prec));
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        // entries read from a file may come from another build: keep them within the fit
        Tune t = it->second.t;
        t.gen_wg = std::min(t.gen_wg, gen_wg_fit(prec, P.S, t.db, false));
        return t;
    }
    if (work_draws < (1u << 20) || !probe) return def;

    // One probe: the full pipeline on the calling problem, best of two timed runs after a
    // warm-up run (the first run warms caches and code).
    auto time_pool = [&](const Tune& t, uint64_t N, uint64_t* keys, double* M, uint64_t cap) {
        double ms = INFINITY;
        for (int rep = 0; rep < 3; ++rep) {
            uint64_t cnt = 0;
            const auto t0 = std::chrono::steady_clock::now();
            const rr_status s = draw_pipeline(P, false, 0x7u, 0, N, RR_MODE_QUANTILE, 1e-4, prec, keys, M, nullptr,
                                              cap, &cnt, st, &t);
            const double dt = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (s != RR_OK) return (double)INFINITY;
            if (rep > 0) ms = std::min(ms, dt);
        }
        return ms;
    };
    // probe pool for the tile and occupancy: ~2^42 MFMA flops, 2^18 .. 2^20 draws; the chunk
    // stage uses 2^23 draws (four chunks of the longest length tried)
    const double ncb = (double)(prec == RR_PREC_GRAM_BF16 ? P.ncb_gram : P.ncb);
    const double flops_per_draw =
        2.0 * 16.0 * (double)P.ks * 32.0 * ncb * (prec == RR_PREC_SPLIT_BF16 || prec == RR_PREC_GRAM_BF16 ? 2.0 : 1.0);
    uint64_t N = (uint64_t)(std::ldexp(1.0, 42) / std::max(1.0, flops_per_draw));
    N = std::min<uint64_t>(std::max<uint64_t>(N, 1u << 18), 1u << 20);
    const uint64_t Nc = 1u << 23;
    const bool chunk_stage = work_draws >= Nc && P.S <= 4;
    const uint64_t cap = (uint64_t)std::ceil(1e-4 * (double)(chunk_stage ? Nc : N)) + 1;
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
            const double ms = time_pool(t, N, keys, M, cap);
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    }
    if (std::isfinite(best_ms) && chunk_stage) {
        double best_c = INFINITY;
        int best_log = best.chunk_log2;
        for (int clog = 19; clog <= 21; ++clog) {
            Tune t = best;
            t.chunk_log2 = clog;
            const double ms = time_pool(t, Nc, keys, M, cap);
            if (ms < best_c) {
                best_c = ms;
                best_log = clog;
            }
        }
        best.chunk_log2 = best_log;
        best_ms = std::isfinite(best_c) ? best_c : best_ms;
    }
    hipFree(keys);
    hipFree(M);
    if (!std::isfinite(best_ms)) return def;
    g_cache[key] = Entry{best, best_ms};
    save_file();
    return best;
}

bool batch_tune_lookup(int prec, int S, Tune* out) {
    if (!tuning_enabled()) return false;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_loaded) load_file();
    auto it = g_cache.find(Key(1, prec, S, -1));
    if (it == g_cache.end()) return false;
    Tune t = it->second.t;
    if (!contract_db_ok(prec, S, t.db)) return false;
    t.gen_wg = std::min(t.gen_wg, gen_wg_fit(prec, S, t.db, true));
    *out = t;
    return true;
}

std::string tune_report() {
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_loaded) load_file();
    return report_json();
}

}  // namespace rr

extern "C" rr_status rr_tune_report(char* buf, uint64_t len, uint64_t* needed) {
    const std::string doc = rr::tune_report();
    if (needed) *needed = doc.size() + 1;
    if (!buf || len < doc.size() + 1) {
        if (buf && len) buf[0] = 0;
        rr::set_error("rr_tune_report: buffer too small");
        return buf ? RR_E_CAPACITY : RR_E_ARG;
    }
    std::memcpy(buf, doc.c_str(), doc.size() + 1);
    return RR_OK;
}
