// Planner: segments a rotation list into HBM passes and builds the device
// tables; executor: enqueues the passes; one-call apply and reductions.
//
// Segmentation (greedy, in application order):
//   * span pass: consecutive rotations whose X masks are repeats of, or
//     linearly independent additions to, a basis of at most `span_m`
//     masks (x = 0 rotations always fit).  Each thread owns one coset of the
//     basis span, so the pass applies them all in registers with one read
//     and one write of the state.
//   * tile pass: consecutive rotations whose X masks lie in a tile frame of
//     B qubits: the low b = B - g qubits plus g "virtual" qubits, each an XOR
//     mask of high (tile-index) bits.  A workgroup holds the 2^g tiles
//     t XOR span(masks) in LDS.  The g = 1 case keeps the two tiles paired by
//     a shared high X part resident, which is the single-GPU form of the
//     common-suffix grouping of Eq. (core); g = 0 holds rotations acting on
//     low qubits only (local operations, Supplementary Methods).
//   * plain pass: a single rotation (pair or diagonal sweep).
// With `commuting` on, a rotation that does not fit may be replaced by a
// later one that does, if that one commutes with every rotation it moves
// ahead of (an exact reordering).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <stdexcept>
#include <string>
#include <vector>

#include "internal.h"
#include "objects.h"

namespace prx {

static inline int popc(uint64_t v) { return __builtin_popcountll(v); }
static inline uint32_t par(uint64_t v) { return (uint32_t)(__builtin_popcountll(v) & 1); }
static inline int hibit(uint64_t v) { return 63 - __builtin_clzll(v); }
static inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static inline bool commute(const KRot &a, const KRot &b) {
    return (popc((a.x & b.z) ^ (a.z & b.x)) & 1) == 0;
}

// Row-echelon basis over GF(2) with pivot = highest set bit of each row;
// every row remembers which of the inserted vectors it combines.
struct Gf2 {
    std::vector<uint64_t> orig;
    std::vector<uint64_t> row, comb;
    // reduce v; returns the remainder and the combination of originals used
    uint64_t reduce(uint64_t v, uint64_t *cmb) const {
        uint64_t c = 0;
        bool again = true;
        while (v && again) {
            again = false;
            for (size_t i = 0; i < row.size(); ++i) {
                if (hibit(row[i]) == hibit(v)) {
                    v ^= row[i];
                    c ^= comb[i];
                    again = true;
                    break;
                }
            }
        }
        if (cmb) *cmb = c;
        return v;
    }
    bool contains(uint64_t v) const { return reduce(v, nullptr) == 0; }
    // adds v (must be independent); returns its index among originals
    size_t add(uint64_t v) {
        uint64_t c;
        uint64_t r = reduce(v, &c);
        const size_t id = orig.size();
        orig.push_back(v);
        row.push_back(r);
        comb.push_back(c ^ (1ull << id));
        return id;
    }
    std::vector<uint32_t> pivots() const {
        std::vector<uint32_t> p;
        for (uint64_t r : row) p.push_back((uint32_t)hibit(r));
        std::sort(p.begin(), p.end());
        return p;
    }
    size_t rank() const { return orig.size(); }
};

// Tau (signed magnitude of i^{nY+1} tan(phi)) and whether it is imaginary.
struct Coef {
    double tau;
    uint32_t imag;
};
static Coef fused_coef(const KRot &r) {
    const double c = std::cos(r.phi), s = std::sin(r.phi);
    const int mq = (popc(r.x & r.z) + 1) & 3;
    Coef o;
    o.tau = ((mq >= 2) ? -1.0 : 1.0) * (s / c);
    o.imag = (uint32_t)(mq & 1);
    return o;
}

// Pending per-slot factors of a chunk (see RotRec): builds the record of a
// rotation in slot `slot` (kSlotDiag for x = 0) with zeta bits `zeta` and
// updates the slot's factor.
struct SlotScale {
    double K[kMaxChunkRank] = {1, 1, 1, 1, 1, 1};
    // m: the chunk's rank (the kernel's coset size 2^m).
    RotRecD record(const KRot &k, uint32_t slot, uint32_t zeta, uint64_t zframe,
                   uint64_t zhigh, int m) {
        const Coef cf = fused_coef(k);
        RotRecD rr;
        rr.z = zframe;
        rr.zhigh = zhigh;
        rr.info = slot | (cf.imag << 4) | (zeta << 8);
        if (m <= kStaticSignRank) {
            uint32_t var = (uint32_t)m << m;  // diagonal
            if (slot != kSlotDiag) {
                const uint32_t zp = (((zeta >> (slot + 1)) << slot) | (zeta & ((1u << slot) - 1u))) &
                                    ((1u << (m - 1)) - 1u);
                var = (slot << m) | (cf.imag << (m - 1)) | zp;
                rr.fold = ((zeta >> slot) & 1u) != 0;
            }
            rr.info |= (var << 16) | (1u << 5);
        }
        if (slot == kSlotDiag) {
            rr.tau_a = cf.tau;
            rr.tau_b = 0.0;
            return rr;
        }
        const double zs = ((zeta >> slot) & 1u) ? -1.0 : 1.0;
        const double kappa = cf.imag ? 1.0 + zs * cf.tau * cf.tau : 1.0 - zs * cf.tau * cf.tau;
        rr.tau_a = cf.tau * K[slot];
        rr.tau_b = cf.tau / (K[slot] * kappa);
        K[slot] *= kappa;
        return rr;
    }
};

static PlainArgs plain_args(int n, const KRot &r) {
    PlainArgs a;
    a.x = r.x;
    a.z = r.z;
    a.n = n;
    a.pivot = r.x ? hibit(r.x) : 0;
    const int nY = popc(r.x & r.z);
    a.nY_odd = nY & 1;
    const int mq = (nY + 1) & 3;
    a.beta_imag = mq & 1;
    a.c = std::cos(r.phi);
    a.beta = ((mq >= 2) ? -1.0 : 1.0) * std::sin(r.phi);
    return a;
}

// ---------------------------------------------------------------- planner

// Coset representatives of a tile chunk: thread t holds k0(t) XOR span(basis)
// with k0(t) = XOR of cvec[i] over the bits i of t, so the cvec must span a
// complement of the basis span (B - m vectors).  LDS serves one access cycle
// for 2^bank_bits consecutive lanes (32 lanes of 8-byte, 16 lanes of 16-byte
// elements); those lanes hit distinct banks when the low bank_bits bits of
// cvec[0 .. bank_bits-1] are independent, so cvec[i] = e_i XOR h with the
// smallest high part h that keeps the set independent (always possible for
// rank m below B - bank_bits), then unit vectors complete the complement.
static void chunk_complement(const Gf2 &basis_span, int B, int nbits, int bank_bits,
                             uint16_t *cvec) {
    Gf2 G = basis_span;
    int t = 0;
    for (int i = 0; i < bank_bits && i < B && t < nbits; ++i) {
        for (uint32_t h = 0; h < (1u << (B - bank_bits)); ++h) {
            const uint32_t c = (1u << i) ^ (h << bank_bits);
            if (!G.contains(c)) {
                G.add(c);
                cvec[t++] = (uint16_t)c;
                break;
            }
        }
    }
    for (int u = 0; u < B && t < nbits; ++u) {
        if (!G.contains(1ull << u)) {
            G.add(1ull << u);
            cvec[t++] = (uint16_t)(1u << u);
        }
    }
}

struct Builder {
    prx_plan &P;
    std::vector<KRot> &R;
    size_t end;
    const PlanCfg &cfg;
    std::vector<RotRecD> recs;  // double records; converted to the dtype at the end

    Builder(prx_plan &p, size_t e) : P(p), R(p.rots), end(e), cfg(p.cfg) {}

    // Length of the span run starting at p (no reordering).
    size_t span_len(size_t p, int mmax) const {
        Gf2 g;
        std::vector<uint64_t> basis;
        size_t j = p;
        const int cap = std::min(cfg.max_fuse, kMaxChunkRots);
        for (; j < end && (int)(j - p) < cap; ++j) {
            const uint64_t x = R[j].x;
            if (x == 0 || std::find(basis.begin(), basis.end(), x) != basis.end()) continue;
            if ((int)basis.size() < mmax && !g.contains(x)) {
                g.add(x);
                basis.push_back(x);
                continue;
            }
            break;
        }
        return j - p;
    }

    bool tile_fits(uint64_t x, int b, Gf2 &M, int g, bool grow) const {
        const uint64_t xh = x >> b;
        if (xh == 0 || M.contains(xh)) return true;
        if ((int)M.rank() < g) {
            if (grow) M.add(xh);
            return true;
        }
        return false;
    }

    size_t tile_len(size_t p, int g) const {
        const int b = cfg.B - g;
        Gf2 M;
        size_t j = p;
        for (; j < end && (int)(j - p) < cfg.max_fuse; ++j)
            if (!tile_fits(R[j].x, b, M, g, true)) break;
        return j - p;
    }

    // With commuting on: bring forward a later rotation that fits, if it
    // commutes with all rotations it jumps over.  `fits` must not mutate.
    template <class F>
    bool pull_forward(size_t j, F fits) {
        if (!cfg.commuting) return false;
        const size_t lim = std::min(end, j + 32);
        for (size_t k = j + 1; k < lim; ++k) {
            if (!fits(R[k])) continue;
            bool ok = true;
            for (size_t i = j; i < k && ok; ++i) ok = commute(R[i], R[k]);
            if (!ok) continue;
            KRot t = R[k];
            for (size_t i = k; i > j; --i) R[i] = R[i - 1];
            R[j] = t;
            return true;
        }
        return false;
    }

    void emit_plain(size_t p) {
        Pass ps;
        ps.kind = kPlain;
        ps.r0 = p;
        ps.r1 = p + 1;
        P.passes.push_back(ps);
        recs.push_back(RotRecD{});
        P.plain_passes++;
    }

    size_t emit_span(size_t p, size_t limit = ~(size_t)0) {
        const size_t stop = std::min(end, limit);
        Gf2 g;
        std::vector<uint64_t> basis;
        size_t j = p;
        auto fits = [&](const KRot &r) {
            if (r.x == 0 || std::find(basis.begin(), basis.end(), r.x) != basis.end()) return true;
            return (int)basis.size() < cfg.span_m && !g.contains(r.x);
        };
        const int cap = std::min(cfg.max_fuse, kMaxChunkRots);
        for (; j < stop && (int)(j - p) < cap; ++j) {
            if (!fits(R[j]) && !pull_forward(j, fits)) break;
            const uint64_t x = R[j].x;
            if (x && std::find(basis.begin(), basis.end(), x) == basis.end()) {
                g.add(x);
                basis.push_back(x);
            }
        }
        if (basis.empty()) {  // diagonal-only run: any direction serves as the basis
            basis.push_back(1ull << (P.n - 1));
            g.add(1ull << (P.n - 1));
        }
        // fixed-rank plans: pad with unused high unit directions
        for (int q = P.n - 1; (int)basis.size() < cfg.pad_rank && q >= 0; --q) {
            if (!g.contains(1ull << q)) {
                g.add(1ull << q);
                basis.push_back(1ull << q);
            }
        }
        Pass ps;
        ps.kind = kSpan;
        ps.r0 = p;
        ps.r1 = j;
        ps.m = (int)basis.size();
        auto piv = g.pivots();
        for (int i = 0; i < ps.m; ++i) {
            ps.basis[i] = basis[i];
            ps.pivot[i] = piv[i];
        }
        double scale = 1.0;
        SlotScale ss;
        for (size_t r = p; r < j; ++r) {
            const KRot &k = R[r];
            scale *= std::cos(k.phi);
            uint32_t slot = kSlotDiag;
            if (k.x) slot = (uint32_t)(std::find(basis.begin(), basis.end(), k.x) - basis.begin());
            uint32_t zeta = 0;
            for (int i = 0; i < ps.m; ++i) zeta |= par(basis[i] & k.z) << i;
            recs.push_back(ss.record(k, slot, zeta, k.z, 0, ps.m));
        }
        for (int i = 0; i < kMaxChunkRank; ++i) ps.fscale[i] = ss.K[i];
        ps.scale = scale;
        P.passes.push_back(ps);
        P.span_passes++;
        return j;
    }

    size_t emit_tile(size_t p, int g, size_t limit = ~(size_t)0) {
        const size_t stop = std::min(end, limit);
        const int b = cfg.B - g;
        const uint64_t low = (b >= 64) ? ~0ull : ((1ull << b) - 1ull);
        Gf2 M;
        size_t j = p;
        auto fits = [&](const KRot &r) {
            Gf2 copy = M;
            return tile_fits(r.x, b, copy, g, false);
        };
        for (; j < stop && (int)(j - p) < cfg.max_fuse; ++j) {
            if (!fits(R[j]) && !pull_forward(j, fits)) break;
            tile_fits(R[j].x, b, M, g, true);
        }
        // Pad the virtual masks to exactly g with unused high unit vectors so
        // that every workgroup holds 2^B amplitudes.
        for (int q = P.n - b - 1; (int)M.rank() < g && q >= 0; --q)
            if (!M.contains(1ull << q)) M.add(1ull << q);
        Pass ps;
        ps.kind = kTile;
        ps.r0 = p;
        ps.r1 = j;
        ps.B = cfg.B;
        ps.b = b;
        ps.g = g;
        ps.m = cfg.m;
        for (int i = 0; i < g; ++i) ps.vmask[i] = M.orig[i];
        auto tp = M.pivots();
        for (int i = 0; i < g; ++i) ps.tpivot[i] = tp[i];
        ps.c0 = P.chunks.size();

        // Map each rotation into the workgroup-local frame (B bits).
        struct Loc {
            uint32_t x, z;
            uint64_t zhigh;
        };
        std::vector<Loc> loc(j - p);
        for (size_t r = p; r < j; ++r) {
            const KRot &k = R[r];
            const uint64_t xh = k.x >> b, zh = k.z >> b;
            uint64_t cmb = 0;
            M.reduce(xh, &cmb);
            uint32_t zv = 0;
            for (int i = 0; i < g; ++i) zv |= par(M.orig[i] & zh) << i;
            Loc L;
            L.x = (uint32_t)(k.x & low) | (uint32_t)(cmb << b);
            L.z = (uint32_t)(k.z & low) | (zv << b);
            L.zhigh = zh;
            loc[r - p] = L;
        }
        // Chunks: runs whose local X masks are repeats of, or independent
        // additions to, a basis of rank <= m.
        double scale = 1.0;
        size_t r = p;
        while (r < j) {
            Gf2 cg;
            std::vector<uint32_t> basis;
            size_t q = r;
            for (; q < j && (int)(q - r) < kMaxChunkRots; ++q) {
                const uint32_t x = loc[q - p].x;
                if (x == 0 || std::find(basis.begin(), basis.end(), x) != basis.end()) continue;
                if ((int)basis.size() < cfg.m && !cg.contains(x)) {
                    cg.add(x);
                    basis.push_back(x);
                    continue;
                }
                break;
            }
            for (int u = cfg.B - 1; (int)basis.size() < cfg.m && u >= 0; --u) {
                if (!cg.contains(1ull << u)) {
                    cg.add(1ull << u);
                    basis.push_back(1u << u);
                }
            }
            ChunkRec ch;
            std::memset(&ch, 0, sizeof(ch));
            ch.rot_begin = (uint32_t)r;
            ch.rot_count = (uint32_t)(q - r);
            for (int i = 0; i < cfg.m; ++i) ch.basis[i] = basis[i];
            chunk_complement(cg, cfg.B, cfg.B - cfg.m, P.dtype == PRX_C64 ? 5 : 4, ch.cvec);
            P.chunks.push_back(ch);
            SlotScale ss;
            for (size_t t = r; t < q; ++t) {
                const KRot &k = R[t];
                const Loc &L = loc[t - p];
                scale *= std::cos(k.phi);
                uint32_t slot = kSlotDiag;
                if (L.x) slot = (uint32_t)(std::find(basis.begin(), basis.end(), L.x) - basis.begin());
                uint32_t zeta = 0;
                for (int i = 0; i < cfg.m; ++i) zeta |= par((uint64_t)basis[i] & L.z) << i;
                recs.push_back(ss.record(k, slot, zeta, L.z, L.zhigh, cfg.m));
            }
            ChunkRec &cb = P.chunks.back();
            for (int i = 0; i < kMaxChunkRank; ++i) cb.fscale[i] = ss.K[i];
            for (int v = 0; v < (1 << cfg.m) && v < 32; ++v) {
                double f = 1.0;
                for (int i = 0; i < cfg.m; ++i)
                    if (v >> i & 1) f *= ss.K[i];
                cb.facd[v] = f;
                cb.facf[v] = (float)f;
            }
            r = q;
        }
        ps.c1 = P.chunks.size();
        ps.scale = scale;
        P.passes.push_back(ps);
        P.tile_passes++;
        return j;
    }

    void run_plain() {
        for (size_t p = P.begin; p < end; ++p) emit_plain(p);
    }

    // Every pass a tile pass (batched tile rounds): from each position the
    // virtual-qubit count that reaches furthest (one virtual qubit always
    // takes at least one rotation).
    void run_tile_only() {
        size_t p = P.begin;
        while (p < end) {
            int gbest = -1;
            size_t best = 0;
            for (int g = 0; g <= cfg.max_virtual && g <= P.n - cfg.B && cfg.B - g >= kMinTileLow;
                 ++g) {
                const size_t f = tile_len(p, g);
                if (f > best) {
                    best = f;
                    gbest = g;
                }
            }
            if (gbest < 0) throw std::runtime_error("tile-only plan: no tile frame fits");
            p = emit_tile(p, gbest);
        }
    }

    void run_span_only() {
        size_t p = P.begin;
        while (p < end) p = emit_span(p);
    }

    // Longest pass from p: its end, the kind (kSpan or kTile) and tile g.
    struct Reach {
        size_t end;
        int kind, g;
    };
    Reach reach_from(size_t p, bool tile_ok) const {
        Reach r{p + span_len(p, cfg.span_m), kSpan, 0};
        if (tile_ok) {
            for (int g = 0; g <= cfg.max_virtual && g <= P.n - cfg.B && cfg.B - g >= kMinTileLow; ++g) {
                const size_t e = p + tile_len(p, g);
                if (e > r.end) r = Reach{e, kTile, g};
            }
        }
        return r;
    }

    // Emits passes covering exactly [p, q): one pass of kind r when it
    // reaches q (always, by construction of r), else further passes.
    void emit_range(size_t p, size_t q, Reach r) {
        while (p < q) {
            if (q - p == 1) {
                emit_plain(p);
                ++p;
                continue;
            }
            size_t got;
            if (r.kind == kTile) {
                // the fewest virtual qubits that still cover [p, q): longer
                // contiguous tiles stream faster
                int g = r.g;
                for (int h = 0; h < r.g; ++h)
                    if (cfg.B - h >= kMinTileLow && p + tile_len(p, h) >= q) {
                        g = h;
                        break;
                    }
                got = emit_tile(p, g, q);
            } else {
                got = emit_span(p, q);
            }
            if (got <= p) {
                emit_plain(p);
                got = p + 1;
            }
            p = got;
            r = Reach{q, kSpan, 0};
        }
    }

    // Minimum number of passes: every pass may end anywhere inside its
    // longest reach (a prefix of a valid pass is valid), so the next pass
    // starts at the cut inside the current reach whose own reach is furthest
    // (the greedy that is optimal for covering a line by jumps).
    void run_fused() {
        const bool tile_ok = P.n >= cfg.B + 1 && tile_supported(P.dtype, cfg.B, cfg.m);
        if (cfg.commuting) {
            run_fused_greedy(tile_ok);
            return;
        }
        const size_t b0 = P.begin;
        std::vector<Reach> reach(end - b0);
        for (size_t p = b0; p < end; ++p) reach[p - b0] = reach_from(p, tile_ok);
        size_t p = b0;
        while (p < end) {
            const Reach &r = reach[p - b0];
            if (r.end >= end) {
                emit_range(p, end, r);
                break;
            }
            size_t cut = r.end, far = reach[r.end - b0].end;
            for (size_t c = p + 1; c < r.end; ++c) {
                if (reach[c - b0].end > far) {
                    far = reach[c - b0].end;
                    cut = c;
                }
            }
            // a span pass covering [p, cut) when one exists (cheaper than a tile pass)
            Reach use = r;
            if (r.kind == kTile && p + span_len(p, cfg.span_m) >= cut) use = Reach{cut, kSpan, 0};
            emit_range(p, cut, use);
            p = cut;
        }
    }

    void run_fused_greedy(bool tile_ok) {
        size_t p = P.begin;
        while (p < end) {
            const size_t fs = span_len(p, cfg.span_m);
            size_t ft = 0;
            int gbest = 0;
            if (tile_ok) {
                for (int g = 0; g <= cfg.max_virtual && g <= P.n - cfg.B && cfg.B - g >= kMinTileLow; ++g) {
                    const size_t f = tile_len(p, g);
                    if (f > ft) {
                        ft = f;
                        gbest = g;
                    }
                }
            }
            if (ft > fs && ft >= 2) {
                p = emit_tile(p, gbest);
            } else {
                const size_t q = emit_span(p);
                if (q - p == 1 && P.passes.back().kind == kSpan) {
                    P.passes.pop_back();
                    P.span_passes--;
                    recs.pop_back();
                    emit_plain(p);
                }
                p = q;
            }
        }
    }
};

}  // namespace prx

using namespace prx;

// ---------------------------------------------------------------- plan API

namespace prx {

void tile_args(int n, const Pass &ps, TileArgs &a) {
    std::memset(&a, 0, sizeof(a));
    for (int k = 0; k < ps.g; ++k) {
        a.vmask[k] = ps.vmask[k];
        a.tpivots |= (uint64_t)(ps.tpivot[k] & 63u) << (6 * k);
    }
    // slot u NT of the tile-set: tile (u NT) >> b, offset (u NT) mod 2^b
    const uint32_t nt = 1u << (ps.B - ps.m);
    for (uint32_t u = 0; u < (1u << ps.m); ++u) {
        const uint32_t v = (u * nt) >> ps.b;
        uint64_t c = 0;
        for (int k = 0; k < ps.g; ++k)
            if (v >> k & 1) c ^= ps.vmask[k];
        a.uoff[u] = (c << ps.b) | ((u * nt) & ((1u << ps.b) - 1u));
    }
    a.n = n;
    a.b = ps.b;
    a.g = ps.g;
    a.chunk_begin = (uint32_t)ps.c0;
    a.chunk_count = (uint32_t)(ps.c1 - ps.c0);
    a.scale = ps.scale;
}

// ------------------------------------------------------------ relabelling
//
// A layout places logical qubit q at index bit phys(q).  The planner only
// uses layouts that exchange low bit j (j < 4) with one other bit ex[j]
// (ex[j] = j: no exchange), so the low bits, whose 16 contiguous amplitudes
// every tile pass keeps in its frame, can hold qubits the next rotations
// act on.  Going from one such layout to another moves at most the 12 bits
// {0..3} U ex_old U ex_new: one relabelling pass (kPerm).
struct Layout {
    uint32_t ex[4] = {0, 1, 2, 3};
    bool identity() const { return ex[0] == 0 && ex[1] == 1 && ex[2] == 2 && ex[3] == 3; }
    uint32_t phys(uint32_t q) const {
        if (q < 4) return ex[q];
        for (uint32_t j = 0; j < 4; ++j)
            if (ex[j] == q) return j;
        return q;
    }
    uint64_t map(uint64_t m) const {
        uint64_t out = 0;
        while (m) {
            const uint32_t q = (uint32_t)__builtin_ctzll(m);
            m &= m - 1;
            out |= 1ull << phys(q);
        }
        return out;
    }
};

// Passes the simple tile model needs for rotations [p, p + count) under a
// layout: b low bits plus up to g virtual directions of the bits above.
static size_t model_passes(const std::vector<KRot> &R, size_t p, size_t count, const Layout &L,
                           int b, int g, int max_fuse, size_t *covered_by = nullptr,
                           size_t pass_limit = ~(size_t)0) {
    size_t passes = 0, j = p;
    const size_t end = std::min(R.size(), p + count);
    while (j < end && passes < pass_limit) {
        Gf2 M;
        size_t k = j;
        for (; k < end && (int)(k - j) < max_fuse; ++k) {
            const uint64_t xh = L.map(R[k].x) >> b;
            if (xh == 0 || M.contains(xh)) continue;
            if ((int)M.rank() < g) {
                M.add(xh);
                continue;
            }
            break;
        }
        j = k;
        ++passes;
    }
    if (covered_by) *covered_by = j - p;
    return passes;
}

// The layout that puts the four qubits most used by the X masks of
// rotations [p, p + window) in the low bits (qubits already low stay).
static Layout hot_layout(const std::vector<KRot> &R, size_t p, size_t window, int n) {
    std::vector<int> cnt(n, 0);
    const size_t end = std::min(R.size(), p + window);
    for (size_t k = p; k < end; ++k)
        for (uint64_t m = R[k].x; m; m &= m - 1) cnt[__builtin_ctzll(m)]++;
    std::vector<uint32_t> q(n);
    for (int i = 0; i < n; ++i) q[i] = (uint32_t)i;
    std::stable_sort(q.begin(), q.end(), [&](uint32_t a, uint32_t b) { return cnt[a] > cnt[b]; });
    bool want[64] = {};
    for (int i = 0; i < 4; ++i) want[q[i]] = true;
    Layout L;
    // low qubits that stay; the others are exchanged with incoming ones
    std::vector<uint32_t> in;
    for (int i = 0; i < 4; ++i)
        if (q[i] >= 4) in.push_back(q[i]);
    size_t t = 0;
    for (uint32_t j = 0; j < 4; ++j)
        if (!want[j] && t < in.size()) L.ex[j] = in[t++];
    return L;
}

// Relabelling pass from layout A to layout B (index bit phys_A(q) moves to
// phys_B(q) for every qubit q).
static Pass perm_pass(int n, const Layout &A, const Layout &B) {
    std::vector<uint32_t> pos = {0, 1, 2, 3};
    auto add = [&](uint32_t v) {
        if (std::find(pos.begin(), pos.end(), v) == pos.end()) pos.push_back(v);
    };
    for (int j = 0; j < 4; ++j) {
        add(A.ex[j]);
        add(B.ex[j]);
    }
    for (uint32_t v = 4; pos.size() < (size_t)kPermBits && v < (uint32_t)n; ++v) add(v);
    std::sort(pos.begin(), pos.end());
    Pass ps;
    ps.kind = kPerm;
    for (int j = 0; j < kPermBits; ++j) ps.ppos[j] = pos[j];
    // the qubit at index bit pos[j] under A
    for (int j = 0; j < kPermBits; ++j) {
        uint32_t q = pos[j];
        if (q < 4)
            q = A.ex[q] == q ? q : A.ex[q];  // logical qubit held at low bit j
        else
            for (uint32_t i = 0; i < 4; ++i)
                if (A.ex[i] == pos[j]) q = i;
        const uint32_t to = B.phys(q);
        ps.pdst[j] = (uint8_t)(std::find(pos.begin(), pos.end(), to) - pos.begin());
    }
    return ps;
}

static void default_cfg(prx_dtype dt, PlanCfg &c) {
    c.B = (dt == PRX_C64) ? 12 : 11;
    c.m = 4;
    c.span_m = 4;
    c.max_fuse = 128;
    c.max_virtual = 8;
    c.renorm_every = (dt == PRX_C64) ? 1 : -1;
    c.commuting = false;
}

static void apply_opts(const prx_plan_opts *o, PlanCfg &c) {
    if (!o) return;
    if (o->tile_qubits) c.B = o->tile_qubits;
    if (o->chunk_rank) c.m = o->chunk_rank;
    if (o->span_max) c.span_m = o->span_max;
    if (o->max_fuse) c.max_fuse = o->max_fuse;
    if (o->max_virtual) c.max_virtual = o->max_virtual < 0 ? 0 : o->max_virtual;
    if (o->renorm_every) c.renorm_every = o->renorm_every;
    if (o->commuting) c.commuting = o->commuting > 0;
    if (o->tile_only) c.tile_only = o->tile_only > 0;
    if (o->relabel) c.relabel = o->relabel > 0;
    if (o->max_grid > 0)
        c.grid_cap = (unsigned)std::min<uint64_t>((uint64_t)o->max_grid, kMaxGridBlocks);
}

// The threaded rotation loop of the complex64 tile chunks reads one record
// with one 32-byte scalar load: z, zhigh, info, pad, tau_a, tau_b.
static_assert(sizeof(RotRec<float>) == 32 && offsetof(RotRec<float>, zhigh) == 8 &&
                  offsetof(RotRec<float>, info) == 16 && offsetof(RotRec<float>, tau_a) == 24 &&
                  offsetof(RotRec<float>, tau_b) == 28,
              "record layout read by the threaded rotation loop");
// The complex128 loop reads 32 bytes (z, zhigh, info, pad, tau_a) and then
// tau_b at byte 32.
static_assert(sizeof(RotRec<double>) == 40 && offsetof(RotRec<double>, info) == 16 &&
                  offsetof(RotRec<double>, tau_a) == 24 && offsetof(RotRec<double>, tau_b) == 32,
              "record layout read by the complex128 threaded rotation loop");

template <typename T>
static void pack_records(prx_plan &P, const std::vector<RotRecD> &recs) {
    P.rot_table.resize(recs.size() * sizeof(RotRec<T>));
    RotRec<T> *out = reinterpret_cast<RotRec<T> *>(P.rot_table.data());
    for (size_t i = 0; i < recs.size(); ++i) {
        RotRec<T> r;
        std::memset(&r, 0, sizeof(r));
        r.z = recs[i].z;
        r.zhigh = recs[i].zhigh;
        r.info = recs[i].info;
        r.tau_a = (T)(recs[i].fold ? -recs[i].tau_a : recs[i].tau_a);
        r.tau_b = (T)recs[i].tau_b;
        out[i] = r;
    }
}

static prx_status plan_create_impl(const prx_sched *sched, int n, prx_dtype dtype, size_t begin,
                                   size_t end, prx_kernel kernel, const prx_plan_opts *opts,
                                   const PlanCfg *internal, prx_plan **out) {
    if (!sched || !out) return fail(PRX_ERR_INVALID, "null pointer");
    if (dtype != PRX_C64 && dtype != PRX_C128) return fail(PRX_ERR_INVALID, "bad dtype");
    if (kernel < PRX_PLAIN || kernel > PRX_AUTO) return fail(PRX_ERR_INVALID, "bad kernel");
    if (n != sched->n) return fail(PRX_ERR_INVALID, "n differs from the schedule's n");
    if (n < 1) return fail(PRX_ERR_INVALID, "n must be >= 1");
    if (n > 40) return fail(PRX_ERR_UNSUPPORTED, "n > 40 does not fit one device");
    if (begin > end || end > sched->x.size()) return fail(PRX_ERR_INVALID, "bad rotation range");
    prx_plan *P = new (std::nothrow) prx_plan;
    if (!P) return fail(PRX_ERR_OOM, "out of host memory");
    try {
        P->n = n;
        P->dtype = dtype;
        P->kernel = kernel;
        P->begin = 0;
        default_cfg(dtype, P->cfg);
        if (kernel == PRX_AUTO) {
            prx_plan_opts t;
            if (tune_lookup(n, dtype, &t)) apply_opts(&t, P->cfg);
        }
        apply_opts(opts, P->cfg);
        if (internal) P->cfg = *internal;
        const bool fused = kernel != PRX_PLAIN;
        if (P->cfg.tile_only && (!fused || n < P->cfg.B)) {
            delete P;
            return fail(PRX_ERR_INVALID, "tile_only needs a fused kernel and n >= tile_qubits");
        }
        if (fused) {
            if (!tile_supported(dtype, P->cfg.B, P->cfg.m) &&
                (P->n > P->cfg.B || P->cfg.tile_only)) {
                delete P;
                return fail(PRX_ERR_UNSUPPORTED, "tile shape (tile_qubits, chunk_rank) not built");
            }
            if (!span_supported(dtype, P->cfg.span_m) || P->cfg.max_virtual > kMaxVirtual ||
                P->cfg.max_fuse < 1 || P->cfg.max_fuse > 4096) {
                delete P;
                return fail(PRX_ERR_INVALID, "bad planner option");
            }
        }
        // Fused plans apply a rotation in k equal pieces, exp(i phi P) =
        // exp(i (phi/k) P)^k, with k the least integer giving |tan(phi/k)| <=
        // 1/sqrt(2): the pair update's kappa then stays in [1/2, 3/2] and
        // every cosine is at least 0.8 in magnitude.
        P->rots.reserve(end - begin);
        const double tmax = 0.70710678118654752, amax = 0.61547970867038734;  // atan(tmax)
        for (size_t j = begin; j < end; ++j) {
            const double phi = sched->phi[j];
            int pieces = 1;
            if (fused && !(std::fabs(std::tan(phi)) <= tmax))
                pieces = (int)std::ceil(std::fabs(phi) / amax);
            const double part = phi / pieces;
            for (int q = 0; q < pieces; ++q) P->rots.push_back(KRot{sched->x[j], sched->z[j], part, j});
        }
        P->end = P->rots.size();
        std::vector<RotRecD> recs;
        const bool relabel = P->cfg.relabel && fused && !P->cfg.span_only &&
                             n >= std::max(P->cfg.B + 2, 14) &&
                             tile_supported(dtype, P->cfg.B, P->cfg.m);
        if (!relabel) {
            Builder bld(*P, P->end);
            // span passes need 2^(n - m) >= 1 cosets; tiny states fall back to plain
            if (P->cfg.span_only)
                bld.run_span_only();
            else if (P->cfg.tile_only)
                bld.run_tile_only();
            else if (!fused || n < 4)
                bld.run_plain();
            else {
                if (P->cfg.span_m > n - 1) P->cfg.span_m = std::max(1, n - 1);
                bld.run_fused();
            }
            recs.swap(bld.recs);
        } else {
            // Segments between relabelling passes.  At a pass boundary of
            // the simple tile model the planner compares the passes needed
            // for the next kRelabelHorizon passes' worth of rotations under
            // the current layout and under the layout that brings the four
            // qubits most used there into the low bits; it relabels when
            // that saves at least kRelabelGain passes (a relabelling pass
            // moves the state once, as a pass does, but runs no rotations).
            if (P->cfg.span_m > n - 1) P->cfg.span_m = std::max(1, n - 1);
            const int g = std::min(P->cfg.max_virtual, P->cfg.B - kMinTileLow);
            const int b = P->cfg.B - g;
            const int mf = P->cfg.max_fuse;
            constexpr size_t kRelabelHorizon = 16, kRelabelGain = 3;
            const std::vector<KRot> logical = P->rots;
            // the layout worth switching to at rotation q, or `cur` itself
            auto better = [&](size_t q, const Layout &cur) {
                size_t cov = 0;
                model_passes(logical, q, P->end - q, cur, b, g, mf, &cov, kRelabelHorizon);
                const size_t hz = std::max<size_t>(cov, 1);
                const Layout hot = hot_layout(logical, q, hz, n);
                if (std::memcmp(hot.ex, cur.ex, sizeof(cur.ex)) == 0) return cur;
                const size_t a = model_passes(logical, q, hz, cur, b, g, mf);
                const size_t h = model_passes(logical, q, hz, hot, b, g, mf);
                return a >= h + kRelabelGain ? hot : cur;
            };
            Layout cur;
            size_t p = 0;
            while (p < P->end) {
                const Layout use = better(p, cur);
                if (std::memcmp(use.ex, cur.ex, sizeof(cur.ex)) != 0) {
                    P->passes.push_back(perm_pass(n, cur, use));
                    cur = use;
                }
                // the segment runs to the next model pass boundary at which
                // relabelling pays
                size_t q = p;
                for (;;) {
                    size_t c1 = 0;
                    model_passes(logical, q, P->end - q, cur, b, g, mf, &c1, 1);
                    q += std::max<size_t>(c1, 1);
                    if (q >= P->end) break;
                    const Layout nx = better(q, cur);
                    if (std::memcmp(nx.ex, cur.ex, sizeof(cur.ex)) != 0) break;
                }
                const size_t seg_end = std::min(q, P->end);
                for (size_t k = p; k < seg_end; ++k) {
                    P->rots[k].x = cur.map(logical[k].x);
                    P->rots[k].z = cur.map(logical[k].z);
                }
                P->begin = p;
                Builder bld(*P, seg_end);
                bld.run_fused();
                recs.insert(recs.end(), bld.recs.begin(), bld.recs.end());
                p = seg_end;
            }
            P->begin = 0;
            if (!cur.identity()) P->passes.push_back(perm_pass(n, cur, Layout{}));
        }
        // renormalisation between consecutive fused passes
        if (dtype == PRX_C64 && P->cfg.renorm_every > 0) {
            int f = 0;
            for (size_t i = 0; i + 1 < P->passes.size(); ++i) {
                Pass &a = P->passes[i];
                Pass &b = P->passes[i + 1];
                if (a.kind == kPlain || a.kind == kPerm) continue;
                ++f;
                if ((b.kind == kSpan || b.kind == kTile) && f % P->cfg.renorm_every == 0) {
                    a.norm_out = true;
                    b.renorm_in = true;
                }
            }
        }
        if (dtype == PRX_C64)
            pack_records<float>(*P, recs);
        else
            pack_records<double>(*P, recs);
        // workspace layout
        size_t maxblocks = 1;
        for (const Pass &ps : P->passes) {
            if (!ps.norm_out) continue;
            const size_t nb = ps.kind == kSpan ? span_blocks(n, ps.m, P->cfg.grid_cap)
                                               : tile_blocks(n, ps.B, P->cfg.grid_cap);
            maxblocks = std::max(maxblocks, nb);
        }
        WsLayout &w = P->ws;
        w.rot_off = 0;
        w.rot_bytes = P->rot_table.size();
        w.chunk_off = align256(w.rot_off + w.rot_bytes + kRecordReadAhead);
        w.chunk_bytes = P->chunks.size() * sizeof(ChunkRec);
        w.part_off = align256(w.chunk_off + w.chunk_bytes);
        w.part_bytes = maxblocks * sizeof(double);
        w.scal_off = align256(w.part_off + w.part_bytes);
        w.scal_bytes = (1 + kRenormStage) * sizeof(double);
        w.total = align256(w.scal_off + w.scal_bytes);
    } catch (const std::bad_alloc &) {
        delete P;
        return fail(PRX_ERR_OOM, "out of host memory");
    } catch (const std::runtime_error &e) {
        delete P;
        return fail(PRX_ERR_INVALID, e.what());
    }
    *out = P;
    return PRX_OK;
}

prx_status plan_create_cfg(const prx_sched *sched, int n, prx_dtype dtype, const PlanCfg &cfg,
                           prx_plan **out) {
    return plan_create_impl(sched, n, dtype, 0, sched ? sched->x.size() : 0, PRX_FUSED, nullptr,
                            &cfg, out);
}

}  // namespace prx

extern "C" {

prx_status prx_plan_create(const prx_sched *sched, int n, prx_dtype dtype, size_t begin,
                           size_t end, prx_kernel kernel, const prx_plan_opts *opts,
                           prx_plan **out) {
    return plan_create_impl(sched, n, dtype, begin, end, kernel, opts, nullptr, out);
}

prx_status prx_plan_get_info(const prx_plan *P, prx_plan_info *o) {
    if (!P || !o) return fail(PRX_ERR_INVALID, "null pointer");
    std::memset(o, 0, sizeof(*o));
    size_t srcs = 0;
    if (!P->rots.empty()) {
        srcs = 1;
        for (size_t i = 1; i < P->rots.size(); ++i) srcs += P->rots[i].src != P->rots[i - 1].src;
    }
    o->rotations = srcs;
    o->kernel_rotations = P->rots.size();
    o->passes = P->passes.size();
    o->plain_passes = P->plain_passes;
    o->span_passes = P->span_passes;
    o->tile_passes = P->tile_passes;
    o->relabel_passes = 0;
    for (const Pass &ps : P->passes) o->relabel_passes += ps.kind == kPerm;
    o->workspace_bytes = P->ws.total;
    o->mean_fuse = P->passes.empty() ? 0.0 : (double)P->rots.size() / (double)P->passes.size();
    o->tile_qubits = P->cfg.B;
    o->chunk_rank = P->cfg.m;
    o->n = P->n;
    o->dtype = (int)P->dtype;
    return PRX_OK;
}

void prx_plan_destroy(prx_plan *P) { delete P; }

prx_status prx_plan_upload(const prx_plan *P, void *ws, size_t ws_bytes, void *stream) {
    if (!P || !ws) return fail(PRX_ERR_INVALID, "null pointer");
    if (ws_bytes < P->ws.total) return fail(PRX_ERR_INVALID, "workspace too small");
    if ((uintptr_t)ws & 255) return fail(PRX_ERR_INVALID, "workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)ws;
    if (P->ws.rot_bytes)
        PRX_HIP(hipMemcpyAsync(base + P->ws.rot_off, P->rot_table.data(), P->ws.rot_bytes,
                               hipMemcpyHostToDevice, s));
    if (P->ws.chunk_bytes)
        PRX_HIP(hipMemcpyAsync(base + P->ws.chunk_off, P->chunks.data(), P->ws.chunk_bytes,
                               hipMemcpyHostToDevice, s));
    return PRX_OK;
}

}  // extern "C"

namespace prx {

// Enqueues the plan; with `ev` non-null, records ev[3i] before pass i,
// ev[3i+1] after its kernel and ev[3i+2] after its hand-off.
static prx_status execute_impl(const prx_plan *P, void *psi, void *ws, size_t ws_bytes,
                               hipStream_t s, hipEvent_t *ev) {
    if (!P || !psi || !ws) return fail(PRX_ERR_INVALID, "null pointer");
    if (ws_bytes < P->ws.total) return fail(PRX_ERR_INVALID, "workspace too small");
    if (((uintptr_t)psi & 15) || ((uintptr_t)ws & 255))
        return fail(PRX_ERR_INVALID, "misaligned state or workspace");
    char *base = (char *)ws;
    const void *rots = base + P->ws.rot_off;
    const ChunkRec *chunks = (const ChunkRec *)(base + P->ws.chunk_off);
    double *part = (double *)(base + P->ws.part_off);
    double *scal = (double *)(base + P->ws.scal_off);
    for (size_t i = 0; i < P->passes.size(); ++i) {
        const Pass &ps = P->passes[i];
        const double *rin = ps.renorm_in ? scal : nullptr;
        double *nout = ps.norm_out ? part : nullptr;
        unsigned blocks = 0;
        hipError_t e = hipSuccess;
        if (ev) PRX_HIP(hipEventRecord(ev[3 * i], s));
        if (ps.kind == kPlain) {
            e = launch_plain(P->dtype, psi, plain_args(P->n, P->rots[ps.r0]), s, P->cfg.grid_cap);
        } else if (ps.kind == kPerm) {
            PermArgs a;
            std::memset(&a, 0, sizeof(a));
            uint32_t dinv[kPermBits];
            for (int j = 0; j < kPermBits; ++j) {
                a.pos[j] = ps.ppos[j];
                dinv[ps.pdst[j]] = (uint32_t)j;
            }
            for (int j = 0; j < kPermBits; ++j) a.inv[j] = (uint16_t)(1u << dinv[j]);
            for (int u = 0; u < 16; ++u) {
                uint32_t v = 0;
                for (int j = 0; j < 4; ++j)
                    if ((u >> j) & 1) v ^= a.inv[8 + j];
                a.ioff[u] = (uint16_t)v;
            }
            a.n = P->n;
            e = launch_permute(P->dtype, psi, a, s, P->cfg.grid_cap);
        } else if (ps.kind == kSpan) {
            SpanArgs a;
            std::memset(&a, 0, sizeof(a));
            for (int k = 0; k < ps.m; ++k) {
                a.basis[k] = ps.basis[k];
                a.pivot[k] = ps.pivot[k];
            }
            a.rot_begin = (uint32_t)ps.r0;
            a.rot_count = (uint32_t)(ps.r1 - ps.r0);
            a.n = P->n;
            a.scale = ps.scale;
            for (int k = 0; k < kMaxChunkRank; ++k) a.fscale[k] = ps.fscale[k];
            e = launch_span(P->dtype, ps.m, psi, a, rots, rin, nout, s, &blocks, P->cfg.grid_cap);
        } else {
            TileArgs a;
            tile_args(P->n, ps, a);
            e = launch_tile(P->dtype, ps.B, ps.m, psi, a, rots, chunks, rin, nout, s, &blocks,
                            P->cfg.grid_cap);
        }
        if (e != hipSuccess) return hip_fail(e, "pass launch");
        if (ev) PRX_HIP(hipEventRecord(ev[3 * i + 1], s));
        if (ps.norm_out) {
            e = launch_renorm_finish(part, blocks, scal, s);
            if (e != hipSuccess) return hip_fail(e, "renorm launch");
        }
        if (ev) PRX_HIP(hipEventRecord(ev[3 * i + 2], s));
    }
    return PRX_OK;
}

}  // namespace prx

prx_status prx_plan_execute(const prx_plan *P, void *psi, void *ws, size_t ws_bytes,
                            void *stream) {
    return execute_impl(P, psi, ws, ws_bytes, (hipStream_t)stream, nullptr);
}

prx_status prx_plan_execute_timed(const prx_plan *P, void *psi, void *ws, size_t ws_bytes,
                                  void *stream, float *pass_ms, float *renorm_ms) {
    if (!P || !pass_ms) return fail(PRX_ERR_INVALID, "null pointer");
    const size_t np = P->passes.size();
    std::vector<hipEvent_t> ev(3 * np, nullptr);
    prx_status st = PRX_OK;
    for (size_t i = 0; i < ev.size() && st == PRX_OK; ++i) {
        hipError_t e = hipEventCreate(&ev[i]);
        if (e != hipSuccess) st = hip_fail(e, "hipEventCreate");
    }
    hipStream_t s = (hipStream_t)stream;
    if (st == PRX_OK) st = execute_impl(P, psi, ws, ws_bytes, s, ev.data());
    if (st == PRX_OK) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    }
    for (size_t i = 0; i < np && st == PRX_OK; ++i) {
        float a = 0.f, b = 0.f;
        hipError_t e = hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[3 * i + 1], ev[3 * i + 2]);
        if (e != hipSuccess) {
            st = hip_fail(e, "hipEventElapsedTime");
            break;
        }
        pass_ms[i] = a;
        if (renorm_ms) renorm_ms[i] = P->passes[i].norm_out ? b : 0.f;
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    return st;
}

extern "C" {

prx_status prx_plan_pass(const prx_plan *P, size_t i, prx_pass_info *o) {
    if (!P || !o) return fail(PRX_ERR_INVALID, "null pointer");
    if (i >= P->passes.size()) return fail(PRX_ERR_INVALID, "pass index out of range");
    const Pass &ps = P->passes[i];
    std::memset(o, 0, sizeof(*o));
    o->kind = ps.kind;
    o->rot_begin = ps.r0;
    o->rot_count = ps.r1 - ps.r0;
    o->chunk_begin = ps.c0;
    o->chunk_count = ps.c1 - ps.c0;
    o->B = ps.B;
    o->b = ps.b;
    o->g = ps.g;
    o->m = ps.m;
    for (int k = 0; k < kMaxChunkRank; ++k) {
        o->basis[k] = ps.basis[k];
        o->pivot[k] = ps.pivot[k];
    }
    for (int k = 0; k < kMaxVirtual; ++k) {
        o->vmask[k] = ps.vmask[k];
        o->tpivot[k] = ps.tpivot[k];
    }
    o->scale = ps.scale;
    for (int k = 0; k < kMaxChunkRank; ++k) o->fscale[k] = ps.fscale[k];
    o->norm_out = ps.norm_out;
    o->renorm_in = ps.renorm_in;
    for (int k = 0; k < kPermBits; ++k) {
        o->perm_pos[k] = ps.ppos[k];
        o->perm_dst[k] = ps.pdst[k];
    }
    if (ps.kind == kPlain) {
        o->grid_blocks = plain_blocks(P->n, P->rots[ps.r0].x == 0, P->cfg.grid_cap);
        o->block_threads = 256;
    } else if (ps.kind == kPerm) {
        o->grid_blocks = permute_blocks(P->n, P->cfg.grid_cap);
        o->block_threads = 256;
    } else if (ps.kind == kSpan) {
        o->grid_blocks = span_blocks(P->n, ps.m, P->cfg.grid_cap);
        o->block_threads = 256;
    } else {
        o->grid_blocks = tile_blocks(P->n, ps.B, P->cfg.grid_cap);
        o->block_threads = 1u << (ps.B - ps.m);
    }
    return PRX_OK;
}

prx_status prx_plan_chunk(const prx_plan *P, size_t i, prx_chunk_info *o) {
    if (!P || !o) return fail(PRX_ERR_INVALID, "null pointer");
    if (i >= P->chunks.size()) return fail(PRX_ERR_INVALID, "chunk index out of range");
    const ChunkRec &c = P->chunks[i];
    std::memset(o, 0, sizeof(*o));
    for (int k = 0; k < kMaxChunkRank; ++k) o->basis[k] = c.basis[k];
    for (int k = 0; k < kMaxTileThreadBits; ++k) o->cvec[k] = c.cvec[k];
    for (int k = 0; k < kMaxChunkRank; ++k) o->fscale[k] = c.fscale[k];
    o->rot_begin = c.rot_begin;
    o->rot_count = c.rot_count;
    return PRX_OK;
}

prx_status prx_plan_rotation(const prx_plan *P, size_t i, prx_rot_info *o) {
    if (!P || !o) return fail(PRX_ERR_INVALID, "null pointer");
    if (i >= P->rots.size()) return fail(PRX_ERR_INVALID, "rotation index out of range");
    const KRot &k = P->rots[i];
    std::memset(o, 0, sizeof(*o));
    o->x = k.x;
    o->z = k.z;
    o->phi = k.phi;
    o->source = k.src;
    if (P->dtype == PRX_C64) {
        const RotRec<float> &r = reinterpret_cast<const RotRec<float> *>(P->rot_table.data())[i];
        o->zframe = r.z;
        o->zhigh = r.zhigh;
        o->slot = r.info & 15u;
        o->imag = (r.info >> 4) & 1u;
        o->zeta = (r.info >> 8) & 0xffu;
        o->var = (r.info >> 16) & 0xffu;
        o->static_sign = (r.info >> 5) & 1u;
        o->tau = r.tau_a;
        o->tau_b = r.tau_b;
    } else {
        const RotRec<double> &r = reinterpret_cast<const RotRec<double> *>(P->rot_table.data())[i];
        o->zframe = r.z;
        o->zhigh = r.zhigh;
        o->slot = r.info & 15u;
        o->imag = (r.info >> 4) & 1u;
        o->zeta = (r.info >> 8) & 0xffu;
        o->var = (r.info >> 16) & 0xffu;
        o->static_sign = (r.info >> 5) & 1u;
        o->tau = r.tau_a;
        o->tau_b = r.tau_b;
    }
    return PRX_OK;
}

size_t prx_workspace_bytes(int n, prx_dtype dtype, const prx_sched *sched, prx_kernel kernel) {
    if (!sched) return 0;
    prx_plan *P = nullptr;
    if (prx_plan_create(sched, n, dtype, 0, sched->x.size(), kernel, nullptr, &P) != PRX_OK)
        return 0;
    const size_t b = P->ws.total;
    prx_plan_destroy(P);
    return b;
}

prx_status prx_apply_range(void *psi, int n, prx_dtype dtype, const prx_sched *sched,
                           size_t begin, size_t end, prx_kernel kernel, void *ws,
                           size_t ws_bytes, void *stream) {
    prx_plan *P = nullptr;
    prx_status st = prx_plan_create(sched, n, dtype, begin, end, kernel, nullptr, &P);
    if (st != PRX_OK) return st;
    st = prx_plan_upload(P, ws, ws_bytes, stream);
    if (st == PRX_OK) st = prx_plan_execute(P, psi, ws, ws_bytes, stream);
    if (st == PRX_OK) {
        hipError_t e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) st = hip_fail(e, "hipStreamSynchronize");
    }
    prx_plan_destroy(P);
    return st;
}

// ------------------------------------------------------------ reductions

size_t prx_reduce_workspace_bytes(int n) {
    (void)n;
    return align256((2 * kReduceBlocks + 8) * sizeof(double));
}

static prx_status check_state(const void *p, int n, prx_dtype dt) {
    if (!p) return fail(PRX_ERR_INVALID, "null state");
    if (n < 1 || n > 40) return fail(PRX_ERR_INVALID, "n must be in [1, 40]");
    if (dt != PRX_C64 && dt != PRX_C128) return fail(PRX_ERR_INVALID, "bad dtype");
    if ((uintptr_t)p & 15) return fail(PRX_ERR_INVALID, "state not 16-byte aligned");
    return PRX_OK;
}

prx_status prx_overlap(const void *psi0, const void *psi, int n, prx_dtype dtype,
                       double out_re_im[2], void *ws, size_t ws_bytes, void *stream) {
    prx_status st = check_state(psi0, n, dtype);
    if (st == PRX_OK) st = check_state(psi, n, dtype);
    if (st != PRX_OK) return st;
    if (!out_re_im || !ws) return fail(PRX_ERR_INVALID, "null pointer");
    if (ws_bytes < prx_reduce_workspace_bytes(n)) return fail(PRX_ERR_INVALID, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    double *w = (double *)ws;
    hipError_t e = launch_overlap(dtype, psi0, psi, n, w, s);
    if (e != hipSuccess) return hip_fail(e, "overlap launch");
    double h[2];
    PRX_HIP(hipMemcpyAsync(h, w + 2 * kReduceBlocks, sizeof(h), hipMemcpyDeviceToHost, s));
    PRX_HIP(hipStreamSynchronize(s));
    out_re_im[0] = h[0];
    out_re_im[1] = h[1];
    return PRX_OK;
}

prx_status prx_norm2(const void *psi, int n, prx_dtype dtype, double *out, void *ws,
                     size_t ws_bytes, void *stream) {
    prx_status st = check_state(psi, n, dtype);
    if (st != PRX_OK) return st;
    if (!out || !ws) return fail(PRX_ERR_INVALID, "null pointer");
    if (ws_bytes < prx_reduce_workspace_bytes(n)) return fail(PRX_ERR_INVALID, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    double *w = (double *)ws;
    hipError_t e = launch_norm2(dtype, psi, n, w, s);
    if (e != hipSuccess) return hip_fail(e, "norm launch");
    double h[2];
    PRX_HIP(hipMemcpyAsync(h, w + 2 * kReduceBlocks, sizeof(h), hipMemcpyDeviceToHost, s));
    PRX_HIP(hipStreamSynchronize(s));
    *out = h[0];
    return PRX_OK;
}

prx_status prx_amplitude(const void *psi, int n, prx_dtype dtype, uint64_t k,
                         double out_re_im[2], void *stream) {
    prx_status st = check_state(psi, n, dtype);
    if (st != PRX_OK) return st;
    if (!out_re_im) return fail(PRX_ERR_INVALID, "null pointer");
    if (k >> n) return fail(PRX_ERR_INVALID, "index out of range");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == PRX_C64) {
        float h[2];
        PRX_HIP(hipMemcpyAsync(h, (const char *)psi + k * 8, 8, hipMemcpyDeviceToHost, s));
        PRX_HIP(hipStreamSynchronize(s));
        out_re_im[0] = h[0];
        out_re_im[1] = h[1];
    } else {
        double h[2];
        PRX_HIP(hipMemcpyAsync(h, (const char *)psi + k * 16, 16, hipMemcpyDeviceToHost, s));
        PRX_HIP(hipStreamSynchronize(s));
        out_re_im[0] = h[0];
        out_re_im[1] = h[1];
    }
    return PRX_OK;
}

prx_status prx_renormalize(void *psi, int n, prx_dtype dtype, void *ws, size_t ws_bytes,
                           void *stream) {
    double nrm = 0.0;
    prx_status st = prx_norm2(psi, n, dtype, &nrm, ws, ws_bytes, stream);
    if (st != PRX_OK) return st;
    if (!(nrm > 0.0) || !std::isfinite(nrm)) return fail(PRX_ERR_INVALID, "state has zero or non-finite norm");
    hipStream_t s = (hipStream_t)stream;
    double *w = (double *)ws;
    const double scale = 1.0 / std::sqrt(nrm);
    PRX_HIP(hipMemcpyAsync(w + 2 * kReduceBlocks + 4, &scale, sizeof(double),
                           hipMemcpyHostToDevice, s));
    hipError_t e = launch_scale(dtype, psi, n, w + 2 * kReduceBlocks + 4, s);
    if (e != hipSuccess) return hip_fail(e, "scale launch");
    PRX_HIP(hipStreamSynchronize(s));
    return PRX_OK;
}

}  // extern "C"
