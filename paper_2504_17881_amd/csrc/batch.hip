// Batched execution of many independent samples (qDRIFT or partially
// randomised draws, circuits of uneven qubit counts).
//
// Samples that hold a tile frame (n >= B: 12 qubits at complex64, 11 at
// complex128) are planned into tile passes only, with up to 8 virtual
// qubits (7 at complex128, every tile keeping 16 contiguous amplitudes): a
// random-order qDRIFT sequence then fuses 2-2.5 times more rotations per HBM
// pass than with spans.  Smaller samples are planned into
// span passes of fixed rank M (the basis padded with unused high
// directions), every pass with the same 2^(n-M) cosets split into Q slices
// of at most kSliceCosets.  Round p applies pass p of every sample that has
// one: one grid-stride kernel over that round's (sample, tile-set) items and
// one over its (sample, slice) items.  Kernel boundaries order the rounds,
// so no workgroup ever waits on another; the whole sequence of round kernels
// is enqueued back to back (and can be captured as one graph).
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
static constexpr int kBatchTileM = 4;
static constexpr int kBatchMaxVirtual = 8;
// Tile rounds launch one workgroup per (sample, tile-set) item up to this
// many (the hardware keeps as many resident as fit and starts the next as
// soon as one ends), striding beyond it.
static constexpr uint64_t kTileGridCap = 1u << 20;
static int batch_tile_qubits(prx_dtype dt) { return dt == PRX_C64 ? 12 : 11; }

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

// State amplitudes addressed as global memory: the states' addresses come
// from the sample tables, and without the address space the compiler would
// use flat accesses, which also count against the LDS/scalar wait counter.
// Non-temporal: every amplitude is read and written once per pass (8 %
// faster on the qDRIFT batch than ordinary loads and stores).
template <typename T>
using V2 = T __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ Cx<T> gload(uint64_t psi, uint64_t i) {
    const V2<T> v =
        __builtin_nontemporal_load(((const __attribute__((address_space(1))) V2<T> *)psi) + i);
    Cx<T> r;
    r.re = v.x;
    r.im = v.y;
    return r;
}
template <typename T>
__device__ __forceinline__ void gstore(uint64_t psi, uint64_t i, const Cx<T> &a) {
    V2<T> v;
    v.x = a.re;
    v.y = a.im;
    __builtin_nontemporal_store(v, ((__attribute__((address_space(1))) V2<T> *)psi) + i);
}
// 16 bytes per lane: G = 16 / sizeof(Cx<T>) consecutive amplitudes from
// amplitude index i (a multiple of G).
template <typename T>
using V16 = T __attribute__((ext_vector_type(16 / sizeof(T))));
template <typename T>
__device__ __forceinline__ V16<T> gload16(uint64_t psi, uint64_t i) {
    return __builtin_nontemporal_load(
        (const __attribute__((address_space(1))) V16<T> *)(psi + i * sizeof(Cx<T>)));
}
template <typename T>
__device__ __forceinline__ void gstore16(uint64_t psi, uint64_t i, const V16<T> &v) {
    __builtin_nontemporal_store(v, (__attribute__((address_space(1))) V16<T> *)(psi + i * sizeof(Cx<T>)));
}

// Round p: items j in [0, prefixQ[active]) over the first `active` sorted
// samples; item j is slice j - prefixQ[k] of sorted sample k.
// The tables arrive as separate __restrict__ arguments: the compiler then
// knows the state stores cannot change them and reads them with scalar
// loads, so the rotation loop's control values stay uniform.
template <typename T>
__global__ void __launch_bounds__(256)
    k_batch_round(const BSample *__restrict__ samples, const BPass *__restrict__ passes,
                  const void *__restrict__ rot_table, const uint64_t *__restrict__ prefixQ,
                  const uint32_t *__restrict__ order, uint32_t p, uint32_t active,
                  uint64_t items) {
    constexpr int M = kBatchRank;
    for (uint64_t j = blockIdx.x; j < items; j += gridDim.x) {
        // last k < active with prefixQ[k] <= j (uniform across the block)
        uint32_t lo = 0, hi = active;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (prefixQ[mid] <= j) lo = mid; else hi = mid;
        }
        const uint32_t s = order[lo];
        const uint64_t q = j - prefixQ[lo];
        const BSample smp = samples[s];
        const BPass ps = passes[smp.pass_begin + p];
        const uint64_t psi = smp.psi;
        const RotRec<T> *rots = reinterpret_cast<const RotRec<T> *>(rot_table) + ps.rot_begin;
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
            for (int v = 0; v < (1 << M); ++v) amp[v] = gload<T>(psi, k0 ^ X[v]);
            apply_rots<T, M>(amp, k0, 0, rots, ps.rot_count);
#pragma unroll
            for (int v = 0; v < (1 << M); ++v) {
                Cx<T> o;
                o.re = amp[v].re * sc[v];
                o.im = amp[v].im * sc[v];
                gstore<T>(psi, k0 ^ X[v], o);
            }
        }
    }
}

// Tile-mode samples: tile passes of fixed (B, M).
struct BTSample {
    uint64_t psi;
    uint32_t nsets;  // 2^(n - B) tile-sets per pass
    uint32_t pass_begin, pass_count;
    uint32_t n;
};

struct BatchTileArgs {
    const BTSample *samples;
    const TileArgs *passes;
    const ChunkRec *chunks;
    const void *rots;
    const uint64_t *prefixW;  // S_t + 1 tile-set counts over the sorted samples
    const uint32_t *order;
};

template <typename T, int B, int M>
__global__ void __launch_bounds__(1 << (B - M))
    k_batch_tile_round(const BTSample *__restrict__ samples, const TileArgs *__restrict__ passes,
                       const ChunkRec *__restrict__ chunks, const void *__restrict__ rot_table,
                       const uint64_t *__restrict__ prefixW, const uint32_t *__restrict__ order,
                       uint32_t p, uint32_t active, uint64_t items) {
    constexpr int NT = 1 << (B - M);
    constexpr int PER = 1 << M;
    __shared__ __align__(16) Cx<T> lds[1 << B];
    unsigned char *lds_raw = reinterpret_cast<unsigned char *>(lds);
    const uint32_t tid = threadIdx.x;
    uint32_t tmask[B - M];
    tile_thread_masks<B - M>(tid, tmask);
    for (uint64_t j = blockIdx.x; j < items; j += gridDim.x) {
        // last k < active with prefixW[k] <= j (uniform across the block)
        uint32_t lo = 0, hi = active;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (prefixW[mid] <= j) lo = mid; else hi = mid;
        }
        const BTSample smp = samples[order[lo]];
        const uint32_t w = (uint32_t)(j - prefixW[lo]);
        const TileArgs *ta = passes + smp.pass_begin + p;
        const uint64_t psi = smp.psi;
        // the set's base tile and this thread's slots (see k_tile)
        const int b = ta->b, g = ta->g;
        uint64_t tb = w;
        for (int i = 0; i < g; ++i) tb = insert_zero64(tb, (uint32_t)(ta->tpivots >> (6 * i)) & 63u);
        // 16-byte groups of G slots: thread tid's group j holds slots
        // G (tid + j NT) .. + G - 1 (see k_tile)
        constexpr int G = 16 / (int)sizeof(Cx<T>);
        constexpr int GPER = PER / G;
        static_assert(sizeof(V16<T>) == 16 && sizeof(V16<T>) == G * sizeof(Cx<T>), "16-byte groups");
        V16<T> *lds_v = reinterpret_cast<V16<T> *>(lds);
        const uint32_t gtid = (uint32_t)G * tid;
        uint64_t c = tb;
        const uint32_t v = gtid >> b;
        for (int i = 0; i < g; ++i)
            if (v >> i & 1) c ^= ta->vmask[i];
        const uint64_t base = (c << b) | (gtid & ((1u << b) - 1u));
        {
            V16<T> r[GPER];
#pragma unroll
            for (int j = 0; j < GPER; ++j) r[j] = gload16<T>(psi, base ^ ta->uoff[G * j]);
#pragma unroll
            for (int j = 0; j < GPER; ++j) lds_v[tid + (uint32_t)j * NT] = r[j];
        }
        __syncthreads();
        tile_chunks<T, B, M>(lds_raw, tmask, tb, chunks + ta->chunk_begin, ta->chunk_count,
                             reinterpret_cast<const RotRec<T> *>(rot_table));
        const T s = (T)ta->scale;
        {
            V16<T> q[GPER];
#pragma unroll
            for (int j = 0; j < GPER; ++j) q[j] = lds_v[tid + (uint32_t)j * NT];
#pragma unroll
            for (int j = 0; j < GPER; ++j) gstore16<T>(psi, base ^ ta->uoff[G * j], q[j] * s);
        }
        __syncthreads();  // the next item overwrites the LDS
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
    std::vector<uint32_t> round_active;  // span samples with a pass in round p
    // tile-mode samples
    std::vector<prx::BTSample> tsamples;
    std::vector<uint32_t> tsrc;  // tile-mode sample -> sample
    std::vector<prx::TileArgs> tpasses;
    std::vector<prx::ChunkRec> tchunks;
    std::vector<uint64_t> tprefix;
    std::vector<uint32_t> torder;
    std::vector<uint32_t> tround_active;
    uint64_t total_items = 0, total_tile_items = 0;
    uint32_t rounds = 0;
    unsigned max_grid = 0;  // 0: the default grid caps
    // workspace layout
    size_t off_samples = 0, off_passes = 0, off_rots = 0, off_prefix = 0, off_order = 0,
           off_tsamples = 0, off_tpasses = 0, off_tchunks = 0, off_tprefix = 0, off_torder = 0,
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
        const int TB = batch_tile_qubits(dtype);
        PlanCfg span_cfg;
        span_cfg.span_only = true;
        span_cfg.pad_rank = kBatchRank;
        span_cfg.span_m = kBatchRank;
        span_cfg.renorm_every = -1;
        span_cfg.max_fuse = 64;
        PlanCfg tile_cfg;
        tile_cfg.tile_only = true;
        tile_cfg.B = TB;
        tile_cfg.m = kBatchTileM;
        tile_cfg.renorm_every = -1;
        tile_cfg.max_fuse = 128;
        tile_cfg.max_virtual = kBatchMaxVirtual;
        // exact reorders: a later rotation that fits the pass's frame and
        // commutes with every rotation it passes joins the pass (10-20 %
        // fewer passes on random-order qDRIFT sequences)
        tile_cfg.commuting = true;
        for (size_t s = 0; s < S; ++s) {
            const bool tile = n[s] >= TB;
            prx_plan *P = nullptr;
            prx_status st = plan_create_cfg(sched[s], n[s], dtype, tile ? tile_cfg : span_cfg, &P);
            if (st != PRX_OK) {
                delete b;
                return st;
            }
            // every sample keeps a BSample (state address and overlap index);
            // a tile-mode sample has no span passes
            BSample sm;
            std::memset(&sm, 0, sizeof(sm));
            sm.n = (uint32_t)n[s];
            sm.ncos = 1ull << (n[s] - kBatchRank);
            sm.Q = (uint32_t)((sm.ncos + kSliceCosets - 1) / kSliceCosets);
            sm.basis_idx = basis_idx[s];
            sm.pass_begin = (uint32_t)b->passes.size();
            const uint32_t rot_base = (uint32_t)(b->rots.size() / rsz);
            if (tile) {
                BTSample ts;
                std::memset(&ts, 0, sizeof(ts));
                ts.n = (uint32_t)n[s];
                ts.nsets = (uint32_t)(1ull << (n[s] - TB));
                ts.pass_begin = (uint32_t)b->tpasses.size();
                ts.pass_count = (uint32_t)P->passes.size();
                const uint32_t chunk_base = (uint32_t)b->tchunks.size();
                for (const Pass &ps : P->passes) {
                    if (ps.kind != kTile || ps.B != TB || ps.m != kBatchTileM) {
                        prx_plan_destroy(P);
                        delete b;
                        return fail(PRX_ERR_UNSUPPORTED, "tile-only plan with another pass kind");
                    }
                    TileArgs ta;
                    tile_args(n[s], ps, ta);
                    ta.chunk_begin += chunk_base;
                    b->tpasses.push_back(ta);
                }
                for (ChunkRec ch : P->chunks) {
                    ch.rot_begin += rot_base;
                    b->tchunks.push_back(ch);
                }
                b->tsamples.push_back(ts);
            } else {
                sm.pass_count = (uint32_t)P->passes.size();
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
            }
            b->rots.insert(b->rots.end(), P->rot_table.begin(), P->rot_table.end());
            b->samples.push_back(sm);
            if (tile) b->tsrc.push_back((uint32_t)s);
            prx_plan_destroy(P);
        }
        // samples sorted by pass count (descending): round p's active samples
        // are a prefix of this order (tile-mode samples sort last with no
        // span passes)
        b->order.resize(S);
        for (size_t s = 0; s < S; ++s) b->order[s] = (uint32_t)s;
        std::stable_sort(b->order.begin(), b->order.end(), [&](uint32_t x, uint32_t y) {
            return b->samples[x].pass_count > b->samples[y].pass_count;
        });
        b->prefixQ.assign(S + 1, 0);
        for (size_t k = 0; k < S; ++k)
            b->prefixQ[k + 1] = b->prefixQ[k] + b->samples[b->order[k]].Q;
        const size_t St = b->tsamples.size();
        b->torder.resize(St);
        for (size_t s = 0; s < St; ++s) b->torder[s] = (uint32_t)s;
        std::stable_sort(b->torder.begin(), b->torder.end(), [&](uint32_t x, uint32_t y) {
            return b->tsamples[x].pass_count > b->tsamples[y].pass_count;
        });
        b->tprefix.assign(St + 1, 0);
        for (size_t k = 0; k < St; ++k)
            b->tprefix[k + 1] = b->tprefix[k] + b->tsamples[b->torder[k]].nsets;
        const uint32_t span_rounds = b->samples[b->order[0]].pass_count;
        const uint32_t tile_rounds = St ? b->tsamples[b->torder[0]].pass_count : 0;
        b->rounds = std::max(span_rounds, tile_rounds);
        b->round_active.assign(b->rounds, 0);
        b->tround_active.assign(b->rounds, 0);
        size_t active = S, tactive = St;
        for (uint32_t p = 0; p < b->rounds; ++p) {
            while (active > 0 && b->samples[b->order[active - 1]].pass_count <= p) --active;
            while (tactive > 0 && b->tsamples[b->torder[tactive - 1]].pass_count <= p) --tactive;
            b->round_active[p] = (uint32_t)active;
            b->tround_active[p] = (uint32_t)tactive;
            b->total_items += b->prefixQ[active];
            b->total_tile_items += b->tprefix[tactive];
        }
        size_t o = 0;
        b->off_samples = o;  o = al256(o + S * sizeof(BSample));
        b->off_passes = o;   o = al256(o + b->passes.size() * sizeof(BPass));
        b->off_rots = o;     o = al256(o + b->rots.size() + kRecordReadAhead);
        b->off_prefix = o;   o = al256(o + b->prefixQ.size() * sizeof(uint64_t));
        b->off_order = o;    o = al256(o + S * sizeof(uint32_t));
        b->off_tsamples = o; o = al256(o + St * sizeof(BTSample));
        b->off_tpasses = o;  o = al256(o + b->tpasses.size() * sizeof(TileArgs));
        b->off_tchunks = o;  o = al256(o + b->tchunks.size() * sizeof(ChunkRec));
        b->off_tprefix = o;  o = al256(o + b->tprefix.size() * sizeof(uint64_t));
        b->off_torder = o;   o = al256(o + St * sizeof(uint32_t));
        b->total = o;
    } catch (const std::bad_alloc &) {
        delete b;
        return fail(PRX_ERR_OOM, "out of host memory");
    }
    *out = b;
    return PRX_OK;
}

size_t prx_batch_workspace_bytes(const prx_batch *b) { return b ? b->total : 0; }

prx_status prx_batch_get_info(const prx_batch *b, prx_batch_info *out) {
    if (!b || !out) return fail(PRX_ERR_INVALID, "null pointer");
    std::memset(out, 0, sizeof(*out));
    out->samples = b->S;
    out->tile_samples = b->tsamples.size();
    out->rounds = b->rounds;
    for (const BSample &s : b->samples) {
        out->passes += s.pass_count;
        out->amp_sweeps += (double)s.pass_count * std::ldexp(1.0, (int)s.n);
    }
    for (const BTSample &s : b->tsamples) {
        out->passes += s.pass_count;
        out->amp_sweeps += (double)s.pass_count * std::ldexp(1.0, (int)s.n);
    }
    return PRX_OK;
}

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
    for (size_t t = 0; t < b->tsamples.size(); ++t) b->tsamples[t].psi = b->samples[b->tsrc[t]].psi;
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
    const size_t St = b->tsamples.size();
    if (St) {
        PRX_HIP(hipMemcpyAsync(w + b->off_tsamples, b->tsamples.data(), St * sizeof(BTSample),
                               hipMemcpyHostToDevice, st));
        PRX_HIP(hipMemcpyAsync(w + b->off_tpasses, b->tpasses.data(),
                               b->tpasses.size() * sizeof(TileArgs), hipMemcpyHostToDevice, st));
        if (!b->tchunks.empty())
            PRX_HIP(hipMemcpyAsync(w + b->off_tchunks, b->tchunks.data(),
                                   b->tchunks.size() * sizeof(ChunkRec), hipMemcpyHostToDevice,
                                   st));
        PRX_HIP(hipMemcpyAsync(w + b->off_tprefix, b->tprefix.data(),
                               b->tprefix.size() * sizeof(uint64_t), hipMemcpyHostToDevice, st));
        PRX_HIP(hipMemcpyAsync(w + b->off_torder, b->torder.data(), St * sizeof(uint32_t),
                               hipMemcpyHostToDevice, st));
    }
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
    BatchTileArgs ta;
    ta.samples = (const BTSample *)(w + b->off_tsamples);
    ta.passes = (const TileArgs *)(w + b->off_tpasses);
    ta.chunks = (const ChunkRec *)(w + b->off_tchunks);
    ta.rots = w + b->off_rots;
    ta.prefixW = (const uint64_t *)(w + b->off_tprefix);
    ta.order = (const uint32_t *)(w + b->off_torder);
    int dev = 0, cus = 256;
    PRX_HIP(hipGetDevice(&dev));
    PRX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    uint64_t cap = (uint64_t)std::max(1, cus) * 8u;
    uint64_t tcap = kTileGridCap;
    if (b->max_grid) {
        cap = std::min<uint64_t>(cap, b->max_grid);
        tcap = std::min<uint64_t>(tcap, b->max_grid);
    }
    const unsigned tile_threads = 1u << (batch_tile_qubits(b->dtype) - kBatchTileM);
    for (uint32_t p = 0; p < b->rounds; ++p) {
        const uint32_t tactive = b->tround_active[p];
        const uint64_t titems = b->tprefix[tactive];
        if (titems) {
            const unsigned grid = (unsigned)std::min<uint64_t>(titems, tcap);
            if (b->dtype == PRX_C64)
                hipLaunchKernelGGL((k_batch_tile_round<float, 12, kBatchTileM>), dim3(grid),
                                   dim3(tile_threads), 0, st, ta.samples, ta.passes, ta.chunks,
                                   ta.rots, ta.prefixW, ta.order, p, tactive, titems);
            else
                hipLaunchKernelGGL((k_batch_tile_round<double, 11, kBatchTileM>), dim3(grid),
                                   dim3(tile_threads), 0, st, ta.samples, ta.passes, ta.chunks,
                                   ta.rots, ta.prefixW, ta.order, p, tactive, titems);
            PRX_HIP(hipGetLastError());
        }
        const uint32_t active = b->round_active[p];
        const uint64_t items = b->prefixQ[active];
        if (items) {
            const unsigned grid = (unsigned)std::min<uint64_t>(items, cap);
            if (b->dtype == PRX_C64)
                hipLaunchKernelGGL(k_batch_round<float>, dim3(grid), dim3(256), 0, st, a.samples,
                                   a.passes, a.rots, a.prefixQ, a.order, p, active, items);
            else
                hipLaunchKernelGGL(k_batch_round<double>, dim3(grid), dim3(256), 0, st, a.samples,
                                   a.passes, a.rots, a.prefixQ, a.order, p, active, items);
            PRX_HIP(hipGetLastError());
        }
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

prx_status prx_batch_set_max_grid(prx_batch *b, unsigned max_grid) {
    if (!b) return fail(PRX_ERR_INVALID, "null batch");
    b->max_grid = max_grid;
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
