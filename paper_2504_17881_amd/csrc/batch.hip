// Batched execution of many independent samples (qDRIFT or partially
// randomised draws, circuits of uneven qubit counts).
//
// Each sample's schedule is planned into span passes of fixed rank M (the
// basis padded with unused high directions), so every pass of a sample has
// the same 2^(n-M) cosets, split into Q slices of at most kSliceCosets.
// Round p applies pass p of every sample that has one: a single grid-stride
// kernel over that round's (sample, slice) items.  Kernel boundaries order
// the rounds, so no workgroup ever waits on another; the whole sequence of
// round kernels is enqueued back to back (and can be captured as one graph).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "device.h"
#include "objects.h"

namespace prx {

static constexpr int kBatchRank = 4;
static constexpr uint64_t kSliceCosets = 8192;

struct BSample {
    uint64_t psi;       // device address of the state
    uint64_t ncos;      // 2^(n - M)
    uint64_t basis_idx; // overlap read-out index
    uint32_t Q;         // slices per pass
    uint32_t pass_begin, pass_count;
    uint32_t n;
};

struct BPass {
    uint64_t basis[kBatchRank];
    uint32_t pivot[kBatchRank];
    uint32_t rot_begin, rot_count;
    double scale;
    double fscale[kBatchRank];
};

struct BatchArgs {
    const BSample *samples;
    const BPass *passes;
    const void *rots;
    const uint64_t *prefixQ;      // S + 1 entries over the pass-count-sorted samples
    const uint32_t *order;        // sorted position -> sample
};

// Round p: items j in [0, prefixQ[active]) over the first `active` sorted
// samples; item j is slice j - prefixQ[k] of sorted sample k.
template <typename T>
__global__ void __launch_bounds__(256) k_batch_round(BatchArgs a, uint32_t p, uint32_t active,
                                                     uint64_t items) {
    constexpr int M = kBatchRank;
    for (uint64_t j = blockIdx.x; j < items; j += gridDim.x) {
        // last k < active with prefixQ[k] <= j (uniform across the block)
        uint32_t lo = 0, hi = active;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.prefixQ[mid] <= j) lo = mid; else hi = mid;
        }
        const uint32_t s = a.order[lo];
        const uint64_t q = j - a.prefixQ[lo];
        const BSample smp = a.samples[s];
        const BPass ps = a.passes[smp.pass_begin + p];
        Cx<T> *psi = reinterpret_cast<Cx<T> *>(smp.psi);
        const RotRec<T> *rots = reinterpret_cast<const RotRec<T> *>(a.rots) + ps.rot_begin;
        uint64_t X[1 << M];
        X[0] = 0;
#pragma unroll
        for (int v = 1; v < (1 << M); ++v) X[v] = X[v & (v - 1)] ^ ps.basis[__builtin_ctz(v)];
        double F[1 << M];
        pending_factors<M>(F, ps.fscale);
        T sc[1 << M];
#pragma unroll
        for (int v = 0; v < (1 << M); ++v) sc[v] = (T)(ps.scale * F[v]);
        const uint64_t c0 = q * kSliceCosets;
        const uint64_t c1 = min(c0 + kSliceCosets, smp.ncos);
        for (uint64_t c = c0 + threadIdx.x; c < c1; c += 256) {
            uint64_t k0 = c;
#pragma unroll
            for (int i = 0; i < M; ++i) k0 = insert_zero64(k0, ps.pivot[i]);
            Cx<T> amp[1 << M];
#pragma unroll
            for (int v = 0; v < (1 << M); ++v) amp[v] = psi[k0 ^ X[v]];
            apply_rots<T, M>(amp, k0, 0, rots, ps.rot_count);
#pragma unroll
            for (int v = 0; v < (1 << M); ++v) {
                Cx<T> o;
                o.re = amp[v].re * sc[v];
                o.im = amp[v].im * sc[v];
                psi[k0 ^ X[v]] = o;
            }
        }
    }
}

template <typename T>
__global__ void k_batch_overlaps(const BSample *samples, uint32_t S, double *out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    const Cx<T> *psi = reinterpret_cast<const Cx<T> *>(samples[i].psi);
    const Cx<T> v = psi[samples[i].basis_idx];
    out[2 * i] = (double)v.re;
    out[2 * i + 1] = (double)v.im;
}

}  // namespace prx

// ------------------------------------------------------------------- host

struct prx_batch {
    size_t S = 0;
    prx_dtype dtype = PRX_C64;
    std::vector<prx::BSample> samples;
    std::vector<prx::BPass> passes;
    std::vector<unsigned char> rots;
    std::vector<uint64_t> prefixQ;
    std::vector<uint32_t> order;
    std::vector<uint32_t> round_active;  // samples with a pass in round p
    uint64_t total_items = 0;
    uint32_t rounds = 0;
    // workspace layout
    size_t off_samples = 0, off_passes = 0, off_rots = 0, off_prefix = 0, off_order = 0,
           total = 0;
};

struct prx_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using namespace prx;

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

extern "C" {

prx_status prx_batch_create(size_t S, const int *n, const prx_sched *const *sched,
                            prx_dtype dtype, const uint64_t *basis_idx, prx_batch **out) {
    if (!out || !n || !sched || !basis_idx) return fail(PRX_ERR_INVALID, "null pointer");
    if (S == 0) return fail(PRX_ERR_INVALID, "S must be positive");
    if (dtype != PRX_C64 && dtype != PRX_C128) return fail(PRX_ERR_INVALID, "bad dtype");
    for (size_t s = 0; s < S; ++s) {
        if (!sched[s]) return fail(PRX_ERR_INVALID, "null schedule");
        if (n[s] < 6 || n[s] > 34) return fail(PRX_ERR_INVALID, "n must be in [6, 34]");
        if (sched[s]->n != n[s]) return fail(PRX_ERR_INVALID, "schedule n differs from n[s]");
        if (basis_idx[s] >> n[s]) return fail(PRX_ERR_INVALID, "basis index out of range");
    }
    prx_batch *b = new (std::nothrow) prx_batch;
    if (!b) return fail(PRX_ERR_OOM, "out of host memory");
    try {
        b->S = S;
        b->dtype = dtype;
        const size_t rsz = dtype == PRX_C64 ? sizeof(RotRec<float>) : sizeof(RotRec<double>);
        PlanCfg cfg;
        cfg.span_only = true;
        cfg.pad_rank = kBatchRank;
        cfg.span_m = kBatchRank;
        cfg.renorm_every = -1;
        cfg.max_fuse = 64;
        for (size_t s = 0; s < S; ++s) {
            prx_plan *P = nullptr;
            prx_status st = plan_create_cfg(sched[s], n[s], dtype, cfg, &P);
            if (st != PRX_OK) {
                delete b;
                return st;
            }
            BSample sm;
            std::memset(&sm, 0, sizeof(sm));
            sm.n = (uint32_t)n[s];
            sm.ncos = 1ull << (n[s] - kBatchRank);
            sm.Q = (uint32_t)((sm.ncos + kSliceCosets - 1) / kSliceCosets);
            sm.basis_idx = basis_idx[s];
            sm.pass_begin = (uint32_t)b->passes.size();
            sm.pass_count = (uint32_t)P->passes.size();
            const uint32_t rot_base = (uint32_t)(b->rots.size() / rsz);
            for (const Pass &ps : P->passes) {
                BPass bp;
                std::memset(&bp, 0, sizeof(bp));
                for (int i = 0; i < kBatchRank; ++i) {
                    bp.basis[i] = ps.basis[i];
                    bp.pivot[i] = ps.pivot[i];
                }
                bp.rot_begin = rot_base + (uint32_t)ps.r0;
                bp.rot_count = (uint32_t)(ps.r1 - ps.r0);
                bp.scale = ps.scale;
                for (int i = 0; i < kBatchRank; ++i) bp.fscale[i] = ps.fscale[i];
                b->passes.push_back(bp);
            }
            b->rots.insert(b->rots.end(), P->rot_table.begin(), P->rot_table.end());
            b->samples.push_back(sm);
            prx_plan_destroy(P);
        }
        // samples sorted by pass count (descending): round p's active samples
        // are a prefix of this order
        b->order.resize(S);
        for (size_t s = 0; s < S; ++s) b->order[s] = (uint32_t)s;
        std::stable_sort(b->order.begin(), b->order.end(), [&](uint32_t x, uint32_t y) {
            return b->samples[x].pass_count > b->samples[y].pass_count;
        });
        b->prefixQ.assign(S + 1, 0);
        for (size_t k = 0; k < S; ++k)
            b->prefixQ[k + 1] = b->prefixQ[k] + b->samples[b->order[k]].Q;
        b->rounds = b->samples[b->order[0]].pass_count;
        b->round_active.assign(b->rounds, 0);
        size_t active = S;
        for (uint32_t p = 0; p < b->rounds; ++p) {
            while (active > 0 && b->samples[b->order[active - 1]].pass_count <= p) --active;
            b->round_active[p] = (uint32_t)active;
            b->total_items += b->prefixQ[active];
        }
        size_t o = 0;
        b->off_samples = o; o = al256(o + S * sizeof(BSample));
        b->off_passes = o;  o = al256(o + b->passes.size() * sizeof(BPass));
        b->off_rots = o;    o = al256(o + b->rots.size());
        b->off_prefix = o;  o = al256(o + b->prefixQ.size() * sizeof(uint64_t));
        b->off_order = o;   o = al256(o + S * sizeof(uint32_t));
        b->total = o;
    } catch (const std::bad_alloc &) {
        delete b;
        return fail(PRX_ERR_OOM, "out of host memory");
    }
    *out = b;
    return PRX_OK;
}

size_t prx_batch_workspace_bytes(const prx_batch *b) { return b ? b->total : 0; }

prx_status prx_batch_upload(prx_batch *b, void *const *psi, void *ws, size_t ws_bytes,
                            void *stream) {
    if (!b || !psi || !ws) return fail(PRX_ERR_INVALID, "null pointer");
    if (ws_bytes < b->total) return fail(PRX_ERR_INVALID, "workspace too small");
    if ((uintptr_t)ws & 255) return fail(PRX_ERR_INVALID, "workspace not 256-byte aligned");
    for (size_t s = 0; s < b->S; ++s) {
        if (!psi[s] || ((uintptr_t)psi[s] & 15))
            return fail(PRX_ERR_INVALID, "null or misaligned state pointer");
        b->samples[s].psi = (uint64_t)(uintptr_t)psi[s];
    }
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    PRX_HIP(hipMemcpyAsync(w + b->off_samples, b->samples.data(), b->S * sizeof(BSample),
                           hipMemcpyHostToDevice, st));
    PRX_HIP(hipMemcpyAsync(w + b->off_passes, b->passes.data(), b->passes.size() * sizeof(BPass),
                           hipMemcpyHostToDevice, st));
    if (!b->rots.empty())
        PRX_HIP(hipMemcpyAsync(w + b->off_rots, b->rots.data(), b->rots.size(),
                               hipMemcpyHostToDevice, st));
    PRX_HIP(hipMemcpyAsync(w + b->off_prefix, b->prefixQ.data(),
                           b->prefixQ.size() * sizeof(uint64_t), hipMemcpyHostToDevice, st));
    PRX_HIP(hipMemcpyAsync(w + b->off_order, b->order.data(), b->S * sizeof(uint32_t),
                           hipMemcpyHostToDevice, st));
    PRX_HIP(hipStreamSynchronize(st));
    return PRX_OK;
}

prx_status prx_batch_execute(const prx_batch *b, void *ws, size_t ws_bytes,
                             double *overlaps_dev, void *stream) {
    if (!b || !ws || !overlaps_dev) return fail(PRX_ERR_INVALID, "null pointer");
    if (ws_bytes < b->total) return fail(PRX_ERR_INVALID, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    char *w = (char *)ws;
    BatchArgs a;
    a.samples = (const BSample *)(w + b->off_samples);
    a.passes = (const BPass *)(w + b->off_passes);
    a.rots = w + b->off_rots;
    a.prefixQ = (const uint64_t *)(w + b->off_prefix);
    a.order = (const uint32_t *)(w + b->off_order);
    int dev = 0, cus = 256;
    PRX_HIP(hipGetDevice(&dev));
    PRX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const uint64_t cap = (uint64_t)std::max(1, cus) * 8u;
    for (uint32_t p = 0; p < b->rounds; ++p) {
        const uint32_t active = b->round_active[p];
        const uint64_t items = b->prefixQ[active];
        const unsigned grid = (unsigned)std::min<uint64_t>(items, cap);
        if (b->dtype == PRX_C64)
            hipLaunchKernelGGL(k_batch_round<float>, dim3(grid), dim3(256), 0, st, a, p, active,
                               items);
        else
            hipLaunchKernelGGL(k_batch_round<double>, dim3(grid), dim3(256), 0, st, a, p, active,
                               items);
        PRX_HIP(hipGetLastError());
    }
    const unsigned rb = (unsigned)((b->S + 255) / 256);
    if (b->dtype == PRX_C64)
        hipLaunchKernelGGL(k_batch_overlaps<float>, dim3(rb), dim3(256), 0, st, a.samples,
                           (uint32_t)b->S, overlaps_dev);
    else
        hipLaunchKernelGGL(k_batch_overlaps<double>, dim3(rb), dim3(256), 0, st, a.samples,
                           (uint32_t)b->S, overlaps_dev);
    PRX_HIP(hipGetLastError());
    return PRX_OK;
}

prx_status prx_batch_check(const prx_batch *b, const void *ws, void *stream) {
    if (!b || !ws) return fail(PRX_ERR_INVALID, "null pointer");
    PRX_HIP(hipStreamSynchronize((hipStream_t)stream));
    PRX_HIP(hipGetLastError());
    return PRX_OK;
}

void prx_batch_destroy(prx_batch *b) { delete b; }

prx_status prx_batch_run(size_t S, void *const *psi, const int *n, const prx_sched *const *sched,
                         prx_dtype dtype, const uint64_t *basis_idx, double *overlaps, void *ws,
                         size_t ws_bytes, void *stream) {
    if (!overlaps) return fail(PRX_ERR_INVALID, "null pointer");
    prx_batch *b = nullptr;
    prx_status st = prx_batch_create(S, n, sched, dtype, basis_idx, &b);
    if (st != PRX_OK) return st;
    // overlaps land after the batch tables in the workspace
    const size_t need = b->total + al256(2 * S * sizeof(double));
    if (ws_bytes < need) {
        prx_batch_destroy(b);
        return fail(PRX_ERR_INVALID, "workspace too small (need prx_batch_workspace_bytes + 16 S)");
    }
    double *ov_dev = (double *)((char *)ws + b->total);
    st = prx_batch_upload(b, psi, ws, ws_bytes, stream);
    if (st == PRX_OK) st = prx_batch_execute(b, ws, ws_bytes, ov_dev, stream);
    if (st == PRX_OK) st = prx_batch_check(b, ws, stream);
    if (st == PRX_OK) {
        hipError_t e = hipMemcpyAsync(overlaps, ov_dev, 2 * S * sizeof(double),
                                      hipMemcpyDeviceToHost, (hipStream_t)stream);
        if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) st = hip_fail(e, "overlap copy");
    }
    prx_batch_destroy(b);
    return st;
}

// ----------------------------------------------------------------- graphs

static prx_status capture_end(hipStream_t st, prx_status body, prx_graph **out) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (body != PRX_OK) {
        if (g) (void)hipGraphDestroy(g);
        return body;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    prx_graph *G = new (std::nothrow) prx_graph;
    if (!G) {
        (void)hipGraphDestroy(g);
        return fail(PRX_ERR_OOM, "out of host memory");
    }
    G->graph = g;
    e = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete G;
        return hip_fail(e, "hipGraphInstantiate");
    }
    *out = G;
    return PRX_OK;
}

prx_status prx_batch_graph(const prx_batch *b, void *ws, size_t ws_bytes, double *overlaps_dev,
                           void *stream, prx_graph **out) {
    if (!out) return fail(PRX_ERR_INVALID, "null pointer");
    if (!stream) return fail(PRX_ERR_INVALID, "capture needs a non-default stream");
    hipStream_t st = (hipStream_t)stream;
    PRX_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    prx_status body = prx_batch_execute(b, ws, ws_bytes, overlaps_dev, stream);
    return capture_end(st, body, out);
}

prx_status prx_plan_graph(const prx_plan *p, void *psi, void *ws, size_t ws_bytes, void *stream,
                          prx_graph **out) {
    if (!out) return fail(PRX_ERR_INVALID, "null pointer");
    if (!stream) return fail(PRX_ERR_INVALID, "capture needs a non-default stream");
    hipStream_t st = (hipStream_t)stream;
    PRX_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    prx_status body = prx_plan_execute(p, psi, ws, ws_bytes, stream);
    return capture_end(st, body, out);
}

prx_status prx_graph_launch(const prx_graph *g, void *stream) {
    if (!g) return fail(PRX_ERR_INVALID, "null graph");
    PRX_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return PRX_OK;
}

void prx_graph_destroy(prx_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
