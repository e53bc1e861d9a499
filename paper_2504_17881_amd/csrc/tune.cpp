// Autotuner: times candidate planner settings (tile qubits and chunk rank of
// the tile kernel, virtual high qubits per tile, fusion depth, span rank) on
// the caller's schedule and state with HIP events, keeps the fastest per
// (arch, n, dtype) in an in-process cache that PRX_AUTO plans read, and
// saves/loads that cache as JSON.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"
#include "objects.h"

namespace prx {

static std::mutex g_mu;
static std::map<std::string, prx_plan_opts> g_cache;

static std::string key(int n, prx_dtype dt) {
    return "gfx950/" + std::to_string(n) + "/" + (dt == PRX_C64 ? "c64" : "c128");
}

bool tune_lookup(int n, prx_dtype dt, prx_plan_opts *out) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key(n, dt));
    if (it == g_cache.end()) return false;
    if (out) *out = it->second;
    return true;
}

void tune_store(int n, prx_dtype dt, const prx_plan_opts &o) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key(n, dt)] = o;
}

static const char *kFields[] = {"tile_qubits", "chunk_rank", "max_fuse", "span_max",
                                "max_virtual", "renorm_every", "commuting", "relabel"};
static constexpr int kNumFields = (int)(sizeof(kFields) / sizeof(kFields[0]));

static int *field(prx_plan_opts &o, int i) {
    int *f[] = {&o.tile_qubits, &o.chunk_rank, &o.max_fuse, &o.span_max,
                &o.max_virtual, &o.renorm_every, &o.commuting, &o.relabel};
    return f[i];
}

// Times one execution of `P` (after one warm-up execution) in ms.
static prx_status time_plan(const prx_plan *P, void *psi, void *ws, size_t ws_bytes,
                            hipStream_t s, float *ms) {
    prx_status st = prx_plan_upload(P, ws, ws_bytes, s);
    if (st != PRX_OK) return st;
    st = prx_plan_execute(P, psi, ws, ws_bytes, s);
    if (st != PRX_OK) return st;
    hipEvent_t a, b;
    PRX_HIP(hipEventCreate(&a));
    PRX_HIP(hipEventCreate(&b));
    PRX_HIP(hipEventRecord(a, s));
    st = prx_plan_execute(P, psi, ws, ws_bytes, s);
    if (st == PRX_OK) {
        PRX_HIP(hipEventRecord(b, s));
        PRX_HIP(hipEventSynchronize(b));
        PRX_HIP(hipEventElapsedTime(ms, a, b));
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return st;
}

}  // namespace prx

using namespace prx;

extern "C" {

prx_status prx_autotune(void *psi, int n, prx_dtype dtype, const prx_sched *sched, void *ws,
                        size_t ws_bytes, void *stream, prx_plan_opts *best_out,
                        int *trials_out) {
    return prx_autotune_progress(psi, n, dtype, sched, ws, ws_bytes, stream, best_out, trials_out,
                                 nullptr, nullptr);
}

prx_status prx_autotune_progress(void *psi, int n, prx_dtype dtype, const prx_sched *sched,
                                 void *ws, size_t ws_bytes, void *stream,
                                 prx_plan_opts *best_out, int *trials_out,
                                 prx_tune_progress_fn progress, void *user) {
    if (!psi || !sched || !ws) return fail(PRX_ERR_INVALID, "null pointer");
    if (dtype != PRX_C64 && dtype != PRX_C128) return fail(PRX_ERR_INVALID, "bad dtype");
    if (sched->n != n) return fail(PRX_ERR_INVALID, "n differs from the schedule's n");
    hipStream_t s = (hipStream_t)stream;
    struct Shape { int B, m; };
    const Shape shapes[] = {{10, 3}, {10, 4}, {11, 4}, {12, 4}, {12, 5}, {13, 4}, {13, 5}, {14, 4}};
    float best_ms = 0.f;
    prx_plan_opts best;
    std::memset(&best, 0, sizeof(best));
    int trials = 0;
    struct Timed {
        prx_plan_opts o;
        float ms;
    };
    std::vector<Timed> timed;
    auto same = [](const prx_plan_opts &a, const prx_plan_opts &b) {
        return std::memcmp(&a, &b, sizeof(a)) == 0;
    };
    auto run = [&](const prx_plan_opts &o) -> prx_status {
        for (const Timed &t : timed)
            if (same(t.o, o)) return PRX_OK;  // already timed
        prx_plan *P = nullptr;
        prx_status st = prx_plan_create(sched, n, dtype, 0, sched->x.size(), PRX_FUSED, &o, &P);
        if (st != PRX_OK) return PRX_OK;  // setting not applicable: skip
        if (o.relabel) {  // same plan as without relabelling: nothing to time
            bool any = false;
            for (const Pass &ps : P->passes) any |= ps.kind == kPerm;
            if (!any) {
                prx_plan_destroy(P);
                return PRX_OK;
            }
        }
        float ms = 0.f;
        if (P->ws.total <= ws_bytes) {
            st = time_plan(P, psi, ws, ws_bytes, s, &ms);
            if (st == PRX_OK) {
                if (progress) progress(&o, ms, user);
                ++trials;
                timed.push_back(Timed{o, ms});
                if (trials == 1 || ms < best_ms) {
                    best_ms = ms;
                    best = o;
                }
            }
        }
        prx_plan_destroy(P);
        return st;
    };
#define PRX_TUNE_RUN(o)                     \
    do {                                    \
        prx_status st_ = run(o);            \
        if (st_ != PRX_OK) return st_;      \
    } while (0)
    // Stage 1: every built tile shape (tile qubits B, chunk rank m) with the
    // most virtual qubits it allows.
    std::vector<Shape> shapes_ok;
    for (const Shape &sh : shapes) {
        if (!tile_supported(dtype, sh.B, sh.m) || n < sh.B + 1) continue;
        shapes_ok.push_back(sh);
        prx_plan_opts o;
        std::memset(&o, 0, sizeof(o));
        o.tile_qubits = sh.B;
        o.chunk_rank = sh.m;
        o.max_virtual = std::min(kMaxVirtual, sh.B - kMinTileLow);
        o.max_fuse = 128;
        o.span_max = 4;
        PRX_TUNE_RUN(o);
    }
    if (shapes_ok.empty()) {  // too small for tiles: span rank only
        for (int r : {2, 3, 4, 5}) {
            prx_plan_opts o;
            std::memset(&o, 0, sizeof(o));
            o.span_max = r;
            PRX_TUNE_RUN(o);
        }
    } else if (trials > 0) {
        // Stage 2: virtual-qubit count for the two fastest shapes.
        std::vector<Timed> st1 = timed;
        std::sort(st1.begin(), st1.end(), [](const Timed &a, const Timed &b) { return a.ms < b.ms; });
        for (size_t k = 0; k < st1.size() && k < 2; ++k)
            for (int g : {1, 2, 3, 5, 8, 10}) {
                prx_plan_opts o = st1[k].o;
                if (o.tile_qubits - g < kMinTileLow) continue;
                o.max_virtual = g;
                PRX_TUNE_RUN(o);
            }
        // Stage 3: fusion depth, span rank and commuting reorders around the best.
        const prx_plan_opts base = best;
        for (int f : {64, 256}) {
            prx_plan_opts o = base;
            o.max_fuse = f;
            PRX_TUNE_RUN(o);
        }
        for (int r : {3, 5}) {
            prx_plan_opts o = best;
            o.span_max = r;
            PRX_TUNE_RUN(o);
        }
        {
            prx_plan_opts o = best;
            o.commuting = 1;
            PRX_TUNE_RUN(o);
        }
        // Stage 4: the best setting with qubit relabelling allowed (timed
        // only when the planner inserts relabelling passes)
        {
            prx_plan_opts o = best;
            o.relabel = 1;
            PRX_TUNE_RUN(o);
        }
    }
#undef PRX_TUNE_RUN
    if (trials == 0) return fail(PRX_ERR_INVALID, "workspace too small for every candidate");
    tune_store(n, dtype, best);
    if (best_out) *best_out = best;
    if (trials_out) *trials_out = trials;
    return PRX_OK;
}

prx_status prx_autotune_lookup(int n, prx_dtype dtype, prx_plan_opts *out) {
    if (!out) return fail(PRX_ERR_INVALID, "null pointer");
    if (!tune_lookup(n, dtype, out)) return fail(PRX_ERR_UNSUPPORTED, "no cached setting");
    return PRX_OK;
}

prx_status prx_autotune_save(const char *path) {
    if (!path) return fail(PRX_ERR_INVALID, "null path");
    std::ostringstream os;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        os << "{";
        bool first = true;
        for (auto &kv : g_cache) {
            os << (first ? "\n" : ",\n") << "  \"" << kv.first << "\": {";
            prx_plan_opts o = kv.second;
            for (int i = 0; i < kNumFields; ++i) os << (i ? ", " : "") << "\"" << kFields[i] << "\": " << *field(o, i);
            os << "}";
            first = false;
        }
        os << "\n}\n";
    }
    std::ofstream f(path);
    if (!f) return fail(PRX_ERR_INVALID, std::string("cannot write ") + path);
    f << os.str();
    return f ? PRX_OK : fail(PRX_ERR_INVALID, std::string("write failed: ") + path);
}

// Reads the flat format written by prx_autotune_save.
prx_status prx_autotune_load(const char *path) {
    if (!path) return fail(PRX_ERR_INVALID, "null path");
    std::ifstream f(path);
    if (!f) return fail(PRX_ERR_INVALID, std::string("cannot read ") + path);
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t pos = 0;
    std::map<std::string, prx_plan_opts> got;
    while (true) {
        const size_t k0 = t.find("\"gfx950/", pos);
        if (k0 == std::string::npos) break;
        const size_t k1 = t.find('"', k0 + 1);
        const size_t b0 = t.find('{', k1);
        const size_t b1 = t.find('}', b0);
        if (k1 == std::string::npos || b0 == std::string::npos || b1 == std::string::npos)
            return fail(PRX_ERR_INVALID, "malformed autotune file");
        const std::string k = t.substr(k0 + 1, k1 - k0 - 1);
        const std::string body = t.substr(b0, b1 - b0);
        prx_plan_opts o;
        std::memset(&o, 0, sizeof(o));
        for (int i = 0; i < kNumFields; ++i) {
            const std::string fk = std::string("\"") + kFields[i] + "\"";
            const size_t p = body.find(fk);
            if (p == std::string::npos) continue;
            const size_t c = body.find(':', p);
            if (c == std::string::npos) return fail(PRX_ERR_INVALID, "malformed autotune file");
            *field(o, i) = std::atoi(body.c_str() + c + 1);
        }
        got[k] = o;
        pos = b1 + 1;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : got) g_cache[kv.first] = kv.second;
    return PRX_OK;
}

}  // extern "C"
