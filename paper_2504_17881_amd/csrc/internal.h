// Internal declarations shared by the host code (sched.cpp, plan.cpp, tune.cpp) and the HIP
// kernels (kernels.hip, batch.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "prx.h"

namespace prx {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
prx_status fail(prx_status st, const std::string &msg);
prx_status hip_fail(hipError_t e, const char *what);

#define PRX_HIP(call)                                                  \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return ::prx::hip_fail(e_, #call);       \
    } while (0)

// ------------------------------------------------------- device tables
//
// One record per rotation of a fused (span or tile) pass.  The rotation
// exp(i phi P) is applied in the factored form
//     new[k] = cos(phi) * ( psi[k] + tau * sigma(k') * psi[k'] ),
// k' = k XOR x, sigma(j) = (-1)^{popcount(j & z)}, tau = i^{nY+1} tan(phi)
// (nY = popcount(x & z)); the cos(phi) factors of a pass are multiplied
// into one scale applied when the pass stores the state.  For x = 0 the
// partner is k itself.
//
// Pair updates run in place: with a = psi[k] (the pair's element whose
// basis bit is clear) and b = psi[k'],
//     a <- a + tau_a s_b b,   then   b <- b + tau_b s_a a   (new a),
// s_a, s_b the signs sigma; for imaginary tau both terms carry a factor i.
// This equals the 2x2 update when b is stored divided by kappa = 1 -/+
// tau^2 and a per-slot factor K is carried: tau_a = tau K, tau_b =
// tau / (K kappa), K <- K kappa.  An element's stored value times the
// product of K over the basis slots set in its coset label is its true
// value; chunks (and span passes) record those K as `fscale`.
//
//   z      : z mask in the frame the kernel indexes (span: global index;
//            tile: workgroup-local index)
//   zhigh  : tile only: z restricted to the tile-index bits, for the sign
//            contributed by the workgroup's base tile
//   info   : bits 0-3  basis slot of x in the chunk (15 = diagonal, x = 0)
//            bit  4    tau is imaginary (nY + 1 odd)
//            bit  5    static-sign variant (chunk rank <= kStaticSignRank)
//            bits 8-15 zeta: bit i = parity(basis_i & z)
//            bits 16-23 variant index (static-sign chunks)
//   tau_a, tau_b : signed magnitudes (real or imaginary parts); for x = 0
//            only tau_a is used (tan(phi))
template <typename T>
struct RotRec {
    uint64_t z;
    uint64_t zhigh;
    uint32_t info;
    uint32_t pad;
    T tau_a;
    T tau_b;
};

static constexpr uint32_t kSlotDiag = 15;
// Chunks of rank up to kStaticSignRank run one compiled variant per
// (slot, imag, sign pattern); their records carry the variant index in
// info bits 16..23 and tau_a multiplied by (-1)^zeta_slot.
static constexpr int kStaticSignRank = 4;
static constexpr int kMaxChunkRank = 6;
// Virtual qubits of a tile pass: at most 10 XOR masks of tile-index bits,
// and at least 16 contiguous amplitudes per tile (128 B at complex64).
static constexpr int kMaxVirtual = 10;
static constexpr int kMinTileLow = 4;
// Readable bytes after a rotation table: the threaded rotation loops load
// the record after the current one (32 bytes at complex64, 40 at
// complex128) before they know whether one follows.
static constexpr size_t kRecordReadAhead = 64;

// Most threads of a tile workgroup (2^(B - m) <= 2^10).
static constexpr int kMaxTileThreadBits = 10;

// A chunk of a tile pass: up to kMaxChunkRank basis directions in the
// workgroup-local frame and a run of rotations whose x masks are basis
// directions (or zero).  Thread t holds the coset k0(t) XOR span(basis),
// k0(t) = XOR of cvec[i] over the bits i set in t; the cvec span a
// complement of the basis span, and the first ones have independent low
// bits so that the lanes of one LDS access cycle use distinct banks.
struct ChunkRec {
    uint32_t rot_begin;
    uint32_t rot_count;
    uint32_t basis[kMaxChunkRank];
    uint16_t cvec[kMaxTileThreadBits];
    double fscale[kMaxChunkRank];  // pending per-slot factors K at the chunk's end
    // element v's factor, the product of fscale over the bits set in v
    // (v < 2^m, m <= 5), in each state precision
    float facf[32];
    double facd[32];
};

// Longest run of rotations in one chunk (bounds the pending factors: with
// tau^2 <= 1/2 each kappa lies in [1/2, 3/2]).
static constexpr int kMaxChunkRots = 64;

// Kernel arguments of a span pass (one chunk in the global frame).
struct SpanArgs {
    uint64_t basis[kMaxChunkRank];
    uint32_t pivot[kMaxChunkRank];
    uint32_t rot_begin, rot_count;
    int n;
    double scale;                  // product of the pass's cosines
    double fscale[kMaxChunkRank];  // pending per-slot factors K
};

// Kernel arguments of a tile pass.
struct TileArgs {
    // Slot s = tid + u NT of the tile-set holds amplitude
    // ((t ^ vc(tid >> b)) << b | (tid & (2^b - 1))) ^ uoff[u], with vc(v) the
    // XOR of the virtual masks selected by v's bits.
    uint64_t uoff[32];  // 2^m entries (tile chunk rank m <= 5)
    uint64_t vmask[kMaxVirtual];  // virtual masks (tile-index space): tile v of a workgroup's
                                  // set is t XOR (the masks selected by the bits of v)
    uint64_t tpivots;             // pivot bits of the masks' echelon form, ascending,
                                  // 6 bits each (pivot i in bits 6i .. 6i+5)
    int n, b, g;
    uint32_t chunk_begin, chunk_count;
    double scale;
};

// Arguments of a single-rotation sweep.
struct PlainArgs {
    uint64_t x, z;
    int n;
    int pivot;       // highest set bit of x (pair kernels)
    int nY_odd;      // popcount(x & z) odd
    int beta_imag;   // beta = i^{nY+1} sin(phi) is imaginary
    double c;        // cos(phi)
    double beta;     // signed magnitude of beta
};

// Arguments of a qubit-relabelling pass: a permutation of the index bits
// at the kPermBits positions pos[0..11] (ascending; pos[j] = j for j < 4,
// the 16 contiguous amplitudes that coalesce one access), all other bits
// fixed.  Group coordinate s in [0, 2^12) has bit j at index bit pos[j];
// the element at input coordinate s moves to output coordinate D(s), which
// has bit dst[j] set for every bit j of s.  The kernel needs, for output
// coordinate s' = t + 256 u (thread t, slot u), the input coordinate
// D^-1(s') = D^-1(t) XOR D^-1(256 u); inv[j] is D^-1 of bit j, and ioff[u]
// = D^-1(256 u) is precomputed on the host.
static constexpr int kPermBits = 12;
struct PermArgs {
    uint32_t pos[kPermBits];
    uint16_t inv[kPermBits];
    uint16_t ioff[16];
    int n;
};

// Autotune cache (tune.cpp), keyed by (arch, n, dtype).
bool tune_lookup(int n, prx_dtype dt, prx_plan_opts *out);
void tune_store(int n, prx_dtype dt, const prx_plan_opts &o);

struct PlanCfg;
// Plan with explicit internal settings (batched plans: span-only, fixed rank).
prx_status plan_create_cfg(const prx_sched *sched, int n, prx_dtype dtype, const PlanCfg &cfg,
                           prx_plan **out);

// ------------------------------------------------------------ launchers
// All enqueue on `stream` and return hipGetLastError() of the launch.
// `cap` limits the workgroups of a launch (at most kMaxGridBlocks); the
// kernels stride over the rest.
hipError_t launch_plain(prx_dtype dt, void *psi, const PlainArgs &a, hipStream_t s,
                        unsigned cap);
hipError_t launch_span(prx_dtype dt, int m, void *psi, const SpanArgs &a, const void *rots,
                       const double *renorm_in, double *norm_out, hipStream_t s,
                       unsigned *blocks_out, unsigned cap);
hipError_t launch_tile(prx_dtype dt, int B, int m, void *psi, const TileArgs &a,
                       const void *rots, const ChunkRec *chunks, const double *renorm_in,
                       double *norm_out, hipStream_t s, unsigned *blocks_out, unsigned cap);
// Qubit relabelling: one pass over the state, in place (every 2^12-element
// group is closed under the permutation).
hipError_t launch_permute(prx_dtype dt, void *psi, const PermArgs &a, hipStream_t s,
                          unsigned cap);
unsigned permute_blocks(int n, unsigned cap);
// partial sums -> 1/sqrt(sum) into scale_out[0]; scale_out[1 .. kRenormStage]
// is stage-1 scratch (two fixed-shape kernels, deterministic)
static constexpr unsigned kRenormStage = 128;
hipError_t launch_renorm_finish(const double *partials, unsigned count, double *scale_out,
                                hipStream_t s);
// Workgroups of one launch: at most kMaxGridBlocks (at 256 threads, 2^30
// work-items, inside a dispatch's 32-bit work-item range); the kernels
// stride over the rest.
static constexpr uint64_t kMaxGridBlocks = 1ull << 22;
unsigned span_blocks(int n, int m, unsigned cap);
unsigned tile_blocks(int n, int B, unsigned cap);
unsigned plain_blocks(int n, bool diag, unsigned cap);
bool span_supported(prx_dtype dt, int m);
bool tile_supported(prx_dtype dt, int B, int m);

// Reductions.  `ws` holds kReduceBlocks * 2 doubles of partials plus 4
// doubles of result.
static constexpr unsigned kReduceBlocks = 1024;
hipError_t launch_overlap(prx_dtype dt, const void *psi0, const void *psi, int n, double *ws,
                          hipStream_t s);
hipError_t launch_norm2(prx_dtype dt, const void *psi, int n, double *ws, hipStream_t s);
hipError_t launch_scale(prx_dtype dt, void *psi, int n, const double *scale_dev,
                        hipStream_t s);

}  // namespace prx
