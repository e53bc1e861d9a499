/*
 * prx.h -- C ABI of the Pauli-rotation state-vector engine for AMD MI355X
 * (gfx950).
 *
 * The library applies long sequences of Pauli rotations exp(i phi P) to a
 * full 2^n complex state held in device memory and returns overlaps
 * <psi0|psi>.  The rotation sequences come from first- and second-order
 * Trotter, qDRIFT and the partially randomised product formula.
 *
 * Conventions (paper, "Software implementation" and Supplementary Methods,
 * "Pauli-string bit representation"):
 *   - Qubit q is bit q of an amplitude index; qubit 0 is the least
 *     significant bit and carries the first tensor factor.
 *   - A Pauli string is a pair of masks (x, z): bit q of x is set iff the
 *     letter on qubit q is X or Y, bit q of z iff it is Y or Z.
 *   - P|j> = i^{popcount(x & z)} (-1)^{popcount(j & z)} |j XOR x>: the
 *     phase counts the Y letters (mod 4) and the sign is taken from the
 *     source index j.
 *   - exp(i phi P) = cos(phi) I + i sin(phi) P.
 *   - A schedule lists rotations in application order: entry 0 acts first.
 *   - Time evolution is exp(+i t H).
 *
 * Memory and ownership:
 *   - States are caller-owned device buffers of 2^n contiguous complex
 *     numbers: interleaved (re, im) float pairs for PRX_C64, double pairs
 *     for PRX_C128.  Amplitude k is basis state |k>.  Base address aligned
 *     to 16 bytes.
 *   - Workspaces are caller-owned device buffers (aligned to 256 bytes)
 *     whose size the library reports.  The library itself never allocates
 *     device memory.
 *   - Streams are hipStream_t values passed as void*; NULL is the default
 *     stream.  Work is enqueued on that stream only.
 *   - Handles (prx_ham, prx_sched, prx_plan) are library-owned host objects,
 *     immutable after creation except where stated, and may be shared by
 *     threads for reading.
 *
 * Errors: every call returns a prx_status; nothing throws or aborts across
 * the ABI.  On failure prx_last_error() describes the cause (thread-local,
 * valid until the next failing call on the same thread).  Outputs are left
 * untouched on failure unless stated.
 */
#ifndef PRX_H
#define PRX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PRX_OK = 0,
    PRX_ERR_INVALID = 1,     /* bad argument: range, null pointer, non-finite value, size */
    PRX_ERR_OOM = 2,         /* host allocation failed */
    PRX_ERR_HIP = 3,         /* a HIP runtime call failed; prx_last_error() has its string */
    PRX_ERR_UNSUPPORTED = 4  /* valid request the library cannot serve (size, dtype, option) */
} prx_status;

typedef enum { PRX_C64 = 1, PRX_C128 = 2 } prx_dtype;

/* Kernel family used by prx_plan_create / prx_apply_range.
 *   PLAIN: one HBM sweep per rotation (pair update, or diagonal when x = 0).
 *   FUSED: several rotations per HBM sweep (span and tile kernels chosen by
 *          the planner), applying exactly the same rotation product.
 *   AUTO:  FUSED with tile size, chunk rank and fusion depth taken from the
 *          autotune cache when it has an entry for (n, dtype). */
typedef enum { PRX_PLAIN = 0, PRX_FUSED = 1, PRX_AUTO = 2 } prx_kernel;

/* Term ordering used when a schedule is built.
 *   NONE:      terms in the order given.
 *   COMMUTING: as NONE; the planner may additionally swap adjacent
 *              commuting rotations, which leaves the product unchanged.
 *   SUFFIX:    the deterministic terms are stably sorted by (x, z) taken as
 *              unsigned integers (lexicographic ordering, Methods "Data
 *              analysis"), which defines a different product formula; the
 *              sorted list is what prx_sched_view returns. */
typedef enum {
    PRX_REORDER_NONE = 0,
    PRX_REORDER_COMMUTING = 1,
    PRX_REORDER_SUFFIX = 2
} prx_reorder;

typedef struct prx_ham prx_ham;
typedef struct prx_sched prx_sched;
typedef struct prx_plan prx_plan;

/* ------------------------------------------------------------------ */
/* Hamiltonian H = sum_l h_l P_l, lambda = sum_l |h_l|                 */
/* (Methods, "Hamiltonian simulation").                                */
/* ------------------------------------------------------------------ */

/* Copies L terms (host arrays x[L], z[L], h[L]).  INVALID if n not in
 * [1, 63], L = 0, a mask has a bit >= n, or an h is not finite. */
prx_status prx_ham_create(int n, size_t L, const uint64_t *x, const uint64_t *z,
                          const double *h, prx_ham **out);
void prx_ham_destroy(prx_ham *ham);
/* lambda = sum |h_l| accumulated left to right in FP64. */
prx_status prx_ham_lambda(const prx_ham *ham, double *out);

/* ------------------------------------------------------------------ */
/* Schedules: rotation lists (x_j, z_j, phi_j) in application order.   */
/* ------------------------------------------------------------------ */

/* First- (order 1, Eq. define-trotter) or second-order (order 2,
 * symmetric: terms forward at delta/2 then reversed at delta/2) Trotter
 * with delta = t / steps; phi = delta * h (order 1) or (delta * h) * 0.5.
 * reorder = SUFFIX sorts the terms first.  INVALID if steps < 1, order not
 * 1 or 2, t not finite. */
prx_status prx_sched_trotter(const prx_ham *ham, int order, double t, int steps,
                             prx_reorder reorder, prx_sched **out);

/* qDRIFT (Methods, "Hamiltonian simulation"): N terms drawn i.i.d. with
 * p_j = |h_j| / lambda, angle sgn(h_j) * ((lambda * t) / N).  Draws use
 * SplitMix64 seeded with `seed`: u = (next >> 11) * 2^-53 picks the first
 * index whose left-to-right FP64 running sum of |h| exceeds u * lambda.
 * INVALID if N < 1 or lambda = 0. */
prx_status prx_sched_qdrift(const prx_ham *ham, double t, size_t N, uint64_t seed,
                            prx_sched **out);

/* Partially randomised product formula (Eq. hamil_split): D = the L_det
 * terms of largest |h| (ties to the lower index; original order, or sorted
 * when reorder = SUFFIX), R = the rest in original order.  Per step
 * (delta = t / steps): D forward at (delta * h) * 0.5, then r_per_step
 * qDRIFT draws from R at sgn(h) * ((lambda_R * delta) / r_per_step), then D
 * reversed at (delta * h) * 0.5.  One SplitMix64 stream for the whole
 * schedule.  INVALID if L_det > L, steps < 1, or R is non-empty with
 * r_per_step = 0. */
prx_status prx_sched_partial(const prx_ham *ham, size_t L_det, double t, int steps,
                             size_t r_per_step, uint64_t seed, prx_reorder reorder,
                             prx_sched **out);

/* Wraps an explicit rotation list (host arrays of length M, copied). */
prx_status prx_sched_from_rotations(int n, size_t M, const uint64_t *x, const uint64_t *z,
                                    const double *phi, prx_sched **out);

/* Borrowed views of a schedule's arrays, valid until prx_sched_destroy. */
prx_status prx_sched_view(const prx_sched *s, int *n, size_t *M, const uint64_t **x,
                          const uint64_t **z, const double **phi);
void prx_sched_destroy(prx_sched *s);

/* ------------------------------------------------------------------ */
/* Plans: a schedule segmented into HBM passes with device tables.     */
/* ------------------------------------------------------------------ */

/* Optional planner settings; zero fields take defaults. */
typedef struct {
    int tile_qubits;     /* qubits held by one workgroup in the tile kernel (default per dtype) */
    int chunk_rank;      /* rotations' X-span rank a thread holds in registers (default 4) */
    int max_fuse;        /* max rotations per tile pass (default 128) */
    int span_max;        /* max rotations per span pass (default: chunk_rank and repeats) */
    int max_virtual;     /* max high-qubit XOR masks gathered into a tile, <= 10; the tile
                            keeps at least 16 contiguous amplitudes (default 8) */
    int renorm_every;    /* C64: renormalise in FP64 every k passes (default 1; -1 = never) */
    int commuting;       /* 1: planner may swap adjacent commuting rotations (default 0) */
    int tile_only;       /* 1: every pass a tile pass, as batched samples of >= tile_qubits
                            qubits are planned (default 0); INVALID with PRX_PLAIN or
                            n < tile_qubits */
    int relabel;         /* 1: fused plans may insert qubit-relabelling passes (kind 3) that
                            bring the qubits the next rotations act on into the low index
                            bits, which every tile pass keeps in its frame; the last pass
                            restores the original order (default 0; needs n >= 14 and
                            n >= tile_qubits + 2, otherwise ignored) */
    int max_grid;        /* workgroups per sweep launch, at most 2^22 (the default); the
                            kernels stride over the remaining cosets or tile-sets */
} prx_plan_opts;

/* Summary of a plan. */
typedef struct {
    size_t rotations;         /* rotations in [begin, end) */
    size_t kernel_rotations;  /* rotations after splitting large angles (fused only) */
    size_t passes;            /* HBM sweeps over the state */
    size_t plain_passes;      /* single-rotation sweeps */
    size_t span_passes;       /* span-kernel sweeps */
    size_t tile_passes;       /* tile-kernel sweeps */
    size_t workspace_bytes;   /* bytes prx_plan_execute needs */
    double mean_fuse;         /* rotations per pass */
    int tile_qubits, chunk_rank;
    int n;                    /* qubits of the state the plan applies to */
    int dtype;                /* prx_dtype of that state */
    size_t relabel_passes;    /* qubit-relabelling sweeps (kind 3) */
} prx_plan_info;

/* Segments rotations [begin, end) of `sched` for a 2^n state of `dtype`
 * with kernel family `kernel`.  Host only; no device calls.  opts may be
 * NULL.  INVALID if begin > end or end > M. UNSUPPORTED if n > 40. */
prx_status prx_plan_create(const prx_sched *sched, int n, prx_dtype dtype, size_t begin,
                           size_t end, prx_kernel kernel, const prx_plan_opts *opts,
                           prx_plan **out);
prx_status prx_plan_get_info(const prx_plan *plan, prx_plan_info *out);
void prx_plan_destroy(prx_plan *plan);

/* Copies the plan's tables into `ws` (device, >= workspace_bytes) on
 * `stream`.  Must precede prx_plan_execute with the same workspace; the
 * tables stay valid until the workspace is overwritten.  The host source
 * stays owned by the plan, so the copy may be asynchronous. */
prx_status prx_plan_upload(const prx_plan *plan, void *ws, size_t ws_bytes, void *stream);

/* Enqueues every pass of the plan on `stream` (asynchronous).  psi is the
 * state (device, 2^n of dtype), ws the uploaded workspace. */
prx_status prx_plan_execute(const prx_plan *plan, void *psi, void *ws, size_t ws_bytes,
                            void *stream);

/* As prx_plan_execute, additionally recording a HIP event before and after
 * every pass kernel and after its renormalisation hand-off, then waiting
 * for the stream.  pass_ms[i] receives the duration of pass i's kernel and
 * renorm_ms[i] (nullable) that of its hand-off (0 when it has none); both
 * are host arrays with one entry per pass. */
prx_status prx_plan_execute_timed(const prx_plan *plan, void *psi, void *ws, size_t ws_bytes,
                                  void *stream, float *pass_ms, float *renorm_ms);

/* Plan inspection (read-only views for tests and tools).
 *
 * Passes: kind 0 = single-rotation sweep, 1 = span pass (one chunk in the
 * global index frame, `basis`/`pivot` valid), 2 = tile pass (workgroup
 * frame of B bits = b low qubits + g virtual qubits; workgroup w holds the
 * tiles t XOR (XOR of vmask[i] over the bits i set in v) for v < 2^g, t = w
 * with zeros inserted at the ascending `tpivot` bits of the tile index;
 * chunks [chunk_begin, +count)), 3 = qubit relabelling (the index bit
 * perm_pos[j] of every amplitude moves to bit perm_pos[perm_dst[j]], in
 * place; bits outside perm_pos stay; the rotations after it carry masks in
 * the new bit order, which the plan's last pass restores).
 * `scale` is the product of the pass's cosines, applied at its store. */
typedef struct {
    int kind;
    size_t rot_begin, rot_count;      /* kernel rotations of the pass */
    size_t chunk_begin, chunk_count;  /* tile passes */
    int B, b, g, m;                   /* tile qubits, low qubits, virtual qubits, rank */
    uint64_t basis[6];                /* span: X-mask basis (global frame) */
    uint32_t pivot[6];                /* span: ascending pivot bits of its echelon form */
    uint64_t vmask[10];               /* tile: virtual masks (tile-index space), g used */
    uint32_t tpivot[10];              /* tile: ascending pivot bits of their echelon form */
    double scale;
    double fscale[6];                 /* span: pending per-slot factors (see prx_rot_info) */
    int norm_out, renorm_in;          /* C64 renormalisation hand-off */
    unsigned grid_blocks;             /* workgroups of the pass's launch (an upper bound for
                                         persistent tile launches, which use the resident
                                         count); the kernels stride over the rest */
    unsigned block_threads;           /* threads per workgroup */
    uint32_t perm_pos[12];            /* relabelling: the moved bit positions (ascending) */
    uint32_t perm_dst[12];            /* relabelling: bit perm_pos[j] -> perm_pos[perm_dst[j]] */
} prx_pass_info;

/* A chunk of a tile pass: basis directions in the workgroup frame; thread t
 * of the workgroup holds the coset k0(t) XOR span(basis) with k0(t) the XOR
 * of cvec[i] over the bits i set in t (cvec[0 .. B-m-1] span a complement
 * of the basis span). */
typedef struct {
    uint32_t basis[6];
    uint32_t cvec[10];
    double fscale[6];                 /* pending per-slot factors at the chunk's end */
    size_t rot_begin, rot_count;
} prx_chunk_info;

/* A kernel rotation: (x, z, phi) as applied, in the index-bit order in
 * force where it runs (relabelled plans: after the preceding relabelling
 * passes); fused plans apply a rotation
 * with |tan phi| > 1/sqrt(2) as k equal pieces), its schedule index, and
 * its record: z in the kernel's frame, the tile-index part zhigh, basis slot
 * (15 = diagonal), whether tau = i^{nY+1} tan(phi) is imaginary, zeta (bit
 * i = parity(basis_i & z)), and the pair-update coefficients.  A pair (a, b)
 * (b = a's partner, basis bit set) is updated in place as a <- a + u tau_a
 * s_b b, then b <- b + u tau_b s_a a (u = 1 or i, s the signs); b is then
 * held divided by kappa = 1 -/+ tau^2, tracked as per-slot factors K
 * (tau_a = tau K, tau_b = tau / (K kappa), K <- K kappa); the true value of
 * the element with coset label v is its stored value times the product of
 * fscale[i] over the bits i set in v.
 *
 * Chunks of rank m <= 4 (static_sign = 1) run one compiled update per
 * variant var = slot 2^m + imag 2^(m-1) + zp (m 2^m for x = 0), zp being
 * zeta with bit `slot` removed; tau is then stored multiplied by
 * (-1)^zeta_slot, and pair (v, v | 2^slot) takes both coefficients times
 * s0 (-1)^parity(c(v) & zp), s0 the sign of the coset representative and
 * c(v) = v with bit `slot` removed. */
typedef struct {
    uint64_t x, z;
    double phi;
    size_t source;
    uint64_t zframe, zhigh;
    uint32_t slot, imag, zeta;
    uint32_t var, static_sign;
    double tau;      /* tau_a as stored (for x = 0: tan(phi)) */
    double tau_b;
} prx_rot_info;

prx_status prx_plan_pass(const prx_plan *plan, size_t i, prx_pass_info *out);
prx_status prx_plan_chunk(const prx_plan *plan, size_t i, prx_chunk_info *out);
prx_status prx_plan_rotation(const prx_plan *plan, size_t i, prx_rot_info *out);

/* ------------------------------------------------------------------ */
/* One-call application and reductions.                                */
/* ------------------------------------------------------------------ */

/* Workspace bytes prx_apply_range needs for the whole schedule. */
size_t prx_workspace_bytes(int n, prx_dtype dtype, const prx_sched *sched, prx_kernel kernel);

/* Plans, uploads and executes rotations [begin, end) on psi, then waits
 * for the stream (the host tables must outlive the copy).  Resuming from
 * any rotation index with a second call gives the same product. */
prx_status prx_apply_range(void *psi, int n, prx_dtype dtype, const prx_sched *sched,
                           size_t begin, size_t end, prx_kernel kernel, void *ws,
                           size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * prx_apply_range, but the plan workspace is a library-owned static device
 * buffer of PRX_STATIC_WS_BYTES per GPU (held until the process ends) in
 * place of a caller workspace.  The call allocates no device memory.
 *   psi    device, 2^n contiguous elements of dtype, updated in place;
 *   stream hipStream_t (NULL = default stream); the call waits for it.
 * INVALID when the plan's workspace (prx_plan_info.workspace_bytes, as
 * prx_workspace_bytes reports for the same range) exceeds the buffer,
 * before any device work; otherwise as prx_apply_range.  Every call on one
 * GPU uses that GPU's one buffer: the library serialises its own calls with
 * a lock, and work that overlaps a call on the same GPU through any other
 * path that uses the buffer would race.  Nothing in the buffer needs to
 * start at zero: each call writes every byte it later reads. */
#define PRX_STATIC_WS_BYTES (64u << 20)
prx_status prx_apply_range_static(void *psi, int n, prx_dtype dtype, const prx_sched *sched,
                                  size_t begin, size_t end, prx_kernel kernel, void *stream);

/* Workspace bytes the reductions need for a 2^n state. */
size_t prx_reduce_workspace_bytes(int n);

/* out_re_im = <psi0|psi> = sum_k conj(psi0[k]) psi[k] (Methods, "Data
 * analysis", the signal g(t)), accumulated in FP64 with compensated
 * per-thread sums and a fixed-shape tree (deterministic).  Synchronises
 * the stream. */
prx_status prx_overlap(const void *psi0, const void *psi, int n, prx_dtype dtype,
                       double out_re_im[2], void *ws, size_t ws_bytes, void *stream);

/* out_re_im = <k|psi> = psi[k] widened to FP64.  Synchronises. */
prx_status prx_amplitude(const void *psi, int n, prx_dtype dtype, uint64_t k,
                         double out_re_im[2], void *stream);

/* out = sum_k |psi[k]|^2 in FP64 (as prx_overlap).  Synchronises. */
prx_status prx_norm2(const void *psi, int n, prx_dtype dtype, double *out, void *ws,
                     size_t ws_bytes, void *stream);

/* psi <- psi / sqrt(norm2(psi)), the scale computed in FP64.  Synchronises. */
prx_status prx_renormalize(void *psi, int n, prx_dtype dtype, void *ws, size_t ws_bytes,
                           void *stream);

/* ------------------------------------------------------------------ */
/* Batched samples: shared round launches.                            */
/* ------------------------------------------------------------------ */

typedef struct prx_batch prx_batch;
typedef struct prx_graph prx_graph;

/* Plans S independent runs: sample s applies sched[s] to its own state
 * (2^n[s] amplitudes of dtype) and reports <basis_idx[s]|psi_s> (the
 * observable of the qDRIFT and partially randomised estimators, Methods).
 * A sample of at least 12 qubits (complex64; 11 for complex128) is
 * segmented into tile passes of that many tile qubits with up to 8 virtual
 * qubits (7 for complex128), bringing a later rotation forward into a pass
 * when it commutes with every rotation it passes (the product is unchanged;
 * only the rounding order differs); a smaller one into span passes of rank 4.  Round p applies pass p
 * of every sample that has one, as one grid-stride kernel over that round's
 * (sample, tile-set) items and one over its (sample, slice) items, so all
 * samples share every launch and no workgroup waits on another.  Host only;
 * no device calls.  INVALID if S = 0, an n[s] is outside [6, 34],
 * sched[s]->n != n[s], or basis_idx[s] >= 2^n[s]. */
prx_status prx_batch_create(size_t S, const int *n, const prx_sched *const *sched,
                            prx_dtype dtype, const uint64_t *basis_idx, prx_batch **out);
size_t prx_batch_workspace_bytes(const prx_batch *b);
/* Summary of a batch plan. */
typedef struct {
    size_t samples;       /* S */
    size_t tile_samples;  /* samples planned into tile passes */
    size_t rounds;        /* largest pass count */
    size_t passes;        /* passes summed over the samples */
    double amp_sweeps;    /* sum over samples of passes * 2^n: each sweep reads and
                             writes every amplitude once (algorithmic bytes
                             = 2 * amp_sweeps * bytes per amplitude) */
} prx_batch_info;
prx_status prx_batch_get_info(const prx_batch *b, prx_batch_info *out);
/* Records the device state pointers psi[s] (host array of S distinct,
 * non-overlapping, 16-byte aligned buffers) and copies the batch tables into
 * `ws`; waits for the copies. */
prx_status prx_batch_upload(prx_batch *b, void *const *psi, void *ws, size_t ws_bytes,
                            void *stream);
/* Enqueues, on `stream`, kernels only: at most two per round (the rounds
 * being the largest pass count among the samples) and the overlap read-out into overlaps_dev
 * (device array of 2*S doubles, (re, im) per sample).  It can therefore be
 * replayed and captured in one graph (prx_batch_graph). */
prx_status prx_batch_execute(const prx_batch *b, void *ws, size_t ws_bytes,
                             double *overlaps_dev, void *stream);
/* Caps the grid of every round launch at max_grid workgroups (0 restores
 * the defaults: 2^20 for the tile rounds, 8 per CU for the span rounds);
 * each launch then strides over the rest of its items.  The results do not
 * depend on the cap.  Takes effect at the next prx_batch_execute or
 * prx_batch_graph.  INVALID for a null batch. */
prx_status prx_batch_set_max_grid(prx_batch *b, unsigned max_grid);
/* Waits for the stream and reports any pending HIP error. */
prx_status prx_batch_check(const prx_batch *b, const void *ws, void *stream);
void prx_batch_destroy(prx_batch *b);

/* One-call form: create, upload, execute, check, copy the 2*S overlaps to
 * the host array `overlaps`, destroy.  ws must hold
 * prx_batch_workspace_bytes + 2*S doubles (rounded up to 256 bytes). */
prx_status prx_batch_run(size_t S, void *const *psi, const int *n,
                         const prx_sched *const *sched, prx_dtype dtype,
                         const uint64_t *basis_idx, double *overlaps, void *ws,
                         size_t ws_bytes, void *stream);

/* HIP graphs of a batch execution or of a plan's pass sequence, captured on
 * `stream` (which must not be the default stream) and instantiated; replay
 * with prx_graph_launch on any stream. */
prx_status prx_batch_graph(const prx_batch *b, void *ws, size_t ws_bytes,
                           double *overlaps_dev, void *stream, prx_graph **out);
prx_status prx_plan_graph(const prx_plan *plan, void *psi, void *ws, size_t ws_bytes,
                          void *stream, prx_graph **out);
prx_status prx_graph_launch(const prx_graph *g, void *stream);
void prx_graph_destroy(prx_graph *g);

/* ------------------------------------------------------------------ */
/* Autotuning.                                                         */
/* ------------------------------------------------------------------ */

/* Times candidate settings of the fused planner on `sched` applied to psi
 * (whose contents are destroyed), and records the fastest for (n, dtype)
 * in the in-process cache used by PRX_AUTO.  The search runs in stages:
 * every built tile shape (tile_qubits, chunk_rank; the shape fixes the
 * workgroup size 2^(tile_qubits - chunk_rank) and the wave layout of a
 * tile-set) with the most virtual qubits it allows; the virtual-qubit count
 * for the two fastest shapes; then max_fuse, span_max and commuting reorders
 * around the best.  Each setting is timed on one execution after a warm-up
 * execution.  trials_out (nullable) receives the number of settings timed.
 * INVALID if no setting's workspace fits ws_bytes.  Synchronises. */
prx_status prx_autotune(void *psi, int n, prx_dtype dtype, const prx_sched *sched, void *ws,
                        size_t ws_bytes, void *stream, prx_plan_opts *best_out,
                        int *trials_out);
/* The same, calling progress(opts, ms, user) after each timed setting
 * (progress may be null). */
typedef void (*prx_tune_progress_fn)(const prx_plan_opts *opts, float ms, void *user);
prx_status prx_autotune_progress(void *psi, int n, prx_dtype dtype, const prx_sched *sched,
                                 void *ws, size_t ws_bytes, void *stream,
                                 prx_plan_opts *best_out, int *trials_out,
                                 prx_tune_progress_fn progress, void *user);
/* Reads/writes the autotune cache as JSON text ({"gfx950/n/dtype": {...}}). */
prx_status prx_autotune_save(const char *path);
prx_status prx_autotune_load(const char *path);
/* Returns the cached settings for (n, dtype), or UNSUPPORTED if absent. */
prx_status prx_autotune_lookup(int n, prx_dtype dtype, prx_plan_opts *out);

/* ------------------------------------------------------------------ */
/* Diagnostics.                                                        */
/* ------------------------------------------------------------------ */

/* Thread-local description of the last failure on this thread. */
const char *prx_last_error(void);
/* Library version string. */
const char *prx_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PRX_H */
