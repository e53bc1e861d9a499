// HIP kernels for gfx950 (CDNA4, wave64): Pauli-rotation sweeps over a
// 2^n complex state in HBM, and FP64 reductions.
//
// A rotation exp(i phi P) with P = (x, z) maps each index pair (k, k ^ x)
// through a 2x2 unitary (paper, "Software implementation": the rotation is a
// direct sum of 2x2 blocks, so (i) a permutation with phases by P and (ii) a
// linear combination):
//     new[k]  = cos(phi) psi[k]  + beta * sigma(k') psi[k']
//     new[k'] = cos(phi) psi[k'] + beta * sigma(k)  psi[k]
// with beta = i^{nY+1} sin(phi), nY = popcount(x & z) (the Y count, mod 4),
// sigma(j) = (-1)^{popcount(j & z)} taken from the source index, and
// sigma(k') = sigma(k) (-1)^{nY} (Supplementary Methods, "Pauli-string bit
// representation").  For x = 0 the rotation is diagonal:
// new[k] = (cos(phi) + i sin(phi) sigma(k)) psi[k].
//
// Kernels:
//   k_plain_pair / k_plain_diag : one rotation per HBM sweep.
//   k_span  : several consecutive rotations per sweep; every thread owns one
//             coset k0 XOR span(x_1..x_m) of the rotations' X masks and keeps
//             its 2^m amplitudes in registers.
//   k_tile  : one workgroup owns a tile-set of 2^B amplitudes (2^g tiles of
//             2^b contiguous amplitudes, g high-qubit XOR masks "virtual
//             qubits") held in LDS; the pass's rotations run in chunks, each
//             chunk gathered per thread as a coset of its X span.  The g = 1
//             case is the single-GPU form of the common-suffix grouping of
//             Eq. (core): all rotations sharing the high part of x are applied
//             while the two partner tiles are resident.
// Fused kernels use the factored update new = cos(phi) (psi + tau sigma
// psi'), tau = beta / cos(phi); a pass multiplies its cosines (and an FP64
// renormalisation factor) into one scale applied at the store.

#include <mutex>

#include "device.h"

namespace prx {

// ----------------------------------------------------------------- plain

// Launch grids are capped at kMaxGridBlocks workgroups (2^30 work-items at
// 256 threads, inside the 32-bit work-item range of a dispatch); the sweep
// kernels stride over the rest of the state.
template <typename T, int U>
__global__ void __launch_bounds__(256) k_plain_pair(Cx<T> *__restrict__ psi, PlainArgs a,
                                                    uint64_t npairs) {
    const T c = (T)a.c;
    const T be = (T)a.beta;
    const uint64_t stride = (uint64_t)gridDim.x * (256u * U);
    for (uint64_t base = (uint64_t)blockIdx.x * (256u * U) + threadIdx.x; base < npairs;
         base += stride) {
        uint64_t k[U], kp[U];
        Cx<T> u[U], w[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint64_t j = base + (uint64_t)i * 256u;
            k[i] = insert_zero64(j < npairs ? j : 0, a.pivot);
            kp[i] = k[i] ^ a.x;
            if (j < npairs) {
                u[i] = psi[k[i]];
                w[i] = psi[kp[i]];
            }
        }
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint64_t j = base + (uint64_t)i * 256u;
            if (j >= npairs) continue;
            const uint32_t sk = parity64(k[i] & a.z);
            const T bk = flip(be, sk ^ (uint32_t)a.nY_odd);  // beta sigma(k'), used for new[k]
            const T bkp = flip(be, sk);                      // beta sigma(k),  used for new[k']
            Cx<T> nu, nw;
            if (a.beta_imag) {
                nu.re = c * u[i].re - bk * w[i].im;
                nu.im = c * u[i].im + bk * w[i].re;
                nw.re = c * w[i].re - bkp * u[i].im;
                nw.im = c * w[i].im + bkp * u[i].re;
            } else {
                nu.re = c * u[i].re + bk * w[i].re;
                nu.im = c * u[i].im + bk * w[i].im;
                nw.re = c * w[i].re + bkp * u[i].re;
                nw.im = c * w[i].im + bkp * u[i].im;
            }
            psi[k[i]] = nu;
            psi[kp[i]] = nw;
        }
    }
}

template <typename T, int U>
__global__ void __launch_bounds__(256) k_plain_diag(Cx<T> *__restrict__ psi, PlainArgs a,
                                                    uint64_t N) {
    const T c = (T)a.c;
    const T s = (T)a.beta;  // beta = i sin(phi) for x = 0
    const uint64_t stride = (uint64_t)gridDim.x * (256u * U);
    for (uint64_t base = (uint64_t)blockIdx.x * (256u * U) + threadIdx.x; base < N;
         base += stride) {
        Cx<T> u[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint64_t k = base + (uint64_t)i * 256u;
            if (k < N) u[i] = psi[k];
        }
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint64_t k = base + (uint64_t)i * 256u;
            if (k >= N) continue;
            const T bs = flip(s, parity64(k & a.z));
            Cx<T> nu;
            nu.re = c * u[i].re - bs * u[i].im;
            nu.im = c * u[i].im + bs * u[i].re;
            psi[k] = nu;
        }
    }
}

// ------------------------------------------------------------------ span

template <typename T, int M>
__global__ void __launch_bounds__(256) k_span(Cx<T> *__restrict__ psi, SpanArgs a,
                                              const RotRec<T> *__restrict__ rots,
                                              const double *__restrict__ renorm_in,
                                              double *__restrict__ norm_out) {
    __shared__ double red[4];
    const uint64_t ncos = 1ull << (a.n - M);
    uint64_t X[1 << M];
    X[0] = 0;
#pragma unroll
    for (int v = 1; v < (1 << M); ++v) X[v] = X[v & (v - 1)] ^ a.basis[__builtin_ctz(v)];
    double sc = a.scale;
    if (renorm_in) sc *= *renorm_in;
    double F[1 << M];
    pending_factors<M>(F, a.fscale);
    double nrm = 0.0;
    // grid-stride over the cosets; every thread of a block runs the same
    // number of iterations (the rotation loop's control stays uniform)
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    for (uint64_t t0 = (uint64_t)blockIdx.x * 256u; t0 < ncos; t0 += stride) {
        const uint64_t t = t0 + threadIdx.x;
        const bool live = t < ncos;
        uint64_t k0 = live ? t : 0;
#pragma unroll
        for (int i = 0; i < M; ++i) k0 = insert_zero64(k0, a.pivot[i]);
        Cx<T> amp[1 << M];
        if (live) {
#pragma unroll
            for (int v = 0; v < (1 << M); ++v) amp[v] = psi[k0 ^ X[v]];
        }
        apply_rots<T, M>(amp, k0, 0, rots + a.rot_begin, a.rot_count);
        if (live) {
            // the thread's 2^M squares, each exact in FP64, summed in FP64
#pragma unroll
            for (int v = 0; v < (1 << M); ++v) {
                const T s = (T)(sc * F[v]);
                Cx<T> o;
                o.re = amp[v].re * s;
                o.im = amp[v].im * s;
                psi[k0 ^ X[v]] = o;
                nrm = fma((double)o.re, (double)o.re, nrm);
                nrm = fma((double)o.im, (double)o.im, nrm);
            }
        }
    }
    if (norm_out) {
        nrm = block_sum<256>(nrm, red);
        if (threadIdx.x == 0) norm_out[blockIdx.x] = nrm;
    }
}

// ------------------------------------------------------------------ tile

// A 128 KiB tile-set (14 qubits at complex64, 13 at complex128) fills most
// of the CU's 160 KiB of LDS, so one workgroup runs per CU; it runs
// persistently, striding over the tile-sets and loading the next one into
// registers while it computes the current one.  Smaller tile-sets run one
// workgroup per tile-set (two to five per CU), which overlaps loads and
// compute across workgroups; with 13-qubit complex64 tile-sets that is 7 %
// faster than the persistent form.
template <typename T, int B>
struct TilePersist {
    static constexpr bool value = (sizeof(Cx<T>) << B) >= (128u << 10);
};

// State access of a tile pass, 16 bytes per lane and instruction: a lane
// moves G = 16 / sizeof(Cx<T>) consecutive amplitudes at once (two at
// complex64, one at complex128; measured 4.5 % faster than one complex64
// amplitude per access for the 14-qubit kernel).  Workgroups that own one
// tile-set stream it with non-temporal loads and stores (each amplitude is
// read and written once per pass; measured 3 % faster with 12-qubit
// tile-sets); the persistent kernel, whose prefetched loads overlap the
// previous set's stores, is faster with ordinary ones (non-temporal: 7 %
// slower).
template <typename T>
struct Group {
    static constexpr int G = 16 / (int)sizeof(Cx<T>);  // amplitudes per access
    typedef T V __attribute__((ext_vector_type(2 * G)));
    static_assert(sizeof(V) == 16 && sizeof(V) == G * sizeof(Cx<T>), "16-byte groups");
};
template <bool NT, typename T>
__device__ __forceinline__ typename Group<T>::V group_load(const Cx<T> *p) {
    typedef typename Group<T>::V V;
    if constexpr (NT)
        return __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
    else
        return *reinterpret_cast<const V *>(p);
}
template <bool NT, typename T>
__device__ __forceinline__ void group_store(Cx<T> *p, const typename Group<T>::V &v) {
    typedef typename Group<T>::V V;
    if constexpr (NT)
        __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
    else
        *reinterpret_cast<V *>(p) = v;
}

// Waves per SIMD that the LDS allows a tile shape (tile-sets per CU x waves
// per set / 4 SIMDs), the occupancy the register allocation is asked to
// keep: five 12-qubit complex64 workgroups per CU need at most 96 registers.
template <typename T, int B, int M>
struct TileWaves {
    static constexpr unsigned sets = (160u << 10) / (sizeof(Cx<T>) << B);
    static constexpr unsigned w = sets * ((1u << (B - M)) / 64u) / 4u;
    static constexpr unsigned value = w < 1 ? 1 : (w > 8 ? 8 : w);
};

template <typename T, int B, int M>
__global__ void __launch_bounds__(1 << (B - M))
    __attribute__((amdgpu_waves_per_eu(TileWaves<T, B, M>::value))) k_tile(Cx<T> *__restrict__ psi, TileArgs a,
                                                      const RotRec<T> *__restrict__ rots,
                                                      const ChunkRec *__restrict__ chunks,
                                                      const double *__restrict__ renorm_in,
                                                      double *__restrict__ norm_out) {
    constexpr int NT = 1 << (B - M);  // threads
    constexpr int PER = 1 << M;       // amplitudes per thread (tile-set 2^B)
    constexpr bool PERSIST = TilePersist<T, B>::value;
    static_assert(PER <= 32 && B - M <= kMaxTileThreadBits, "tile shape");
    // The tile-set is the only LDS allocation (2^B amplitudes): 160 KB hold
    // five 12-qubit complex64 workgroups per CU.  Static, so that its address
    // is a link-time constant and LDS addresses are plain byte offsets.
    __shared__ __align__(16) Cx<T> lds[1 << B];
    unsigned char *lds_raw = reinterpret_cast<unsigned char *>(lds);
    const uint32_t tid = threadIdx.x;
    const uint32_t nsets = (uint32_t)(1ull << (a.n - B));

    // Tile v of set w has tile index t(w) ^ vc(v), vc(v) = XOR of the masks
    // selected by v's bits; t(w) inserts zeros at the masks' pivots.  Slot
    // s = G tid + u NT (u = G j) has disjoint thread and u bits, so its
    // global index splits into a per-thread part and the host's uniform
    // uoff[u] (the global offset of slot u NT).
    // HBM traffic moves groups of G slots: thread tid's group j holds slots
    // G (tid + j NT) .. + G - 1, contiguous in memory (b >= 4 low bits).
    constexpr int G = Group<T>::G;
    constexpr int GPER = PER / G;  // groups per thread
    typedef typename Group<T>::V V;
    V *lds_v = reinterpret_cast<V *>(lds);
    const uint32_t gtid = (uint32_t)G * tid;  // the thread's first slot
    const uint64_t vt = [&] {
        uint64_t c = 0;
        const uint32_t v = gtid >> a.b;
        for (int i = 0; i < a.g; ++i)
            if (v >> i & 1) c ^= a.vmask[i];
        return c;
    }();
    // (pivots unpacked with shifts: no indexed load from the argument block)
    auto tile_of = [&](uint32_t w) {
        uint64_t t = w;
        for (int i = 0; i < a.g; ++i) t = insert_zero64(t, (uint32_t)(a.tpivots >> (6 * i)) & 63u);
        return t;
    };
    auto base_of = [&](uint64_t t) { return ((t ^ vt) << a.b) | (gtid & ((1u << a.b) - 1u)); };

    uint32_t tmask[B - M];
    tile_thread_masks<B - M>(tid, tmask);

    double sc = a.scale;
    if (renorm_in) sc *= *renorm_in;
    const T s = (T)sc;
    double nrm = 0.0;

    // Set order: persistent workgroups stride over the sets; otherwise the
    // workgroups, dispatched round-robin over the 8 XCDs, give each XCD a
    // contiguous range of sets (and stride over the rest when the grid is
    // capped: the set count is then a multiple of the grid).
    uint32_t w = blockIdx.x;
    if (!PERSIST && (gridDim.x & 7u) == 0u)
        w = (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
    // Every thread issues all its loads before the first LDS store.  A
    // persistent workgroup enters each iteration with its set in LDS, loads
    // the next set into registers, computes and stores the current one, and
    // only then writes the loaded set to LDS: the loads' wait then sits
    // behind the stores in the same iteration, and the stores drain while
    // the next set is computed.
    // group j of the thread sits at offset uoff[G j] from its base
    V r[GPER];
    auto load_set = [&](uint64_t b0) {
#pragma unroll
        for (int j = 0; j < GPER; ++j) r[j] = group_load<!PERSIST>(psi + (b0 ^ a.uoff[G * j]));
    };
    auto stage_set = [&] {
#pragma unroll
        for (int j = 0; j < GPER; ++j) lds_v[tid + (uint32_t)j * NT] = r[j];
    };
    if (PERSIST && w < nsets) {
        load_set(base_of(tile_of(w)));
        stage_set();
        __syncthreads();
    }
    for (; w < nsets; w += gridDim.x) {
        const uint64_t tb = tile_of(w);
        const uint64_t base = base_of(tb);
        if (!PERSIST) {
            // one set per iteration (several when the grid is capped); a
            // thread writes only the slots it read in the previous store
            // epilogue, so no barrier is needed before the staging
            load_set(base);
            stage_set();
            __syncthreads();
        }
        const uint32_t wn = w + gridDim.x;
        const bool next = PERSIST && wn < nsets;
        if (next) load_set(base_of(tile_of(wn)));

        tile_chunks<T, B, M>(lds_raw, tmask, tb, chunks + a.chunk_begin, a.chunk_count, rots);

        {
            V q[GPER];
#pragma unroll
            for (int j = 0; j < GPER; ++j) q[j] = lds_v[tid + (uint32_t)j * NT];
            // the thread's squares, each exact in FP64, summed in FP64
#pragma unroll
            for (int j = 0; j < GPER; ++j) {
                const V o = q[j] * s;
                group_store<!PERSIST>(psi + (base ^ a.uoff[G * j]), o);
#pragma unroll
                for (int c = 0; c < 2 * G; ++c) nrm = fma((double)o[c], (double)o[c], nrm);
            }
        }
        if (next) {
            // the staging writes exactly the slots this thread read in the
            // store epilogue above (LDS operations of a wave stay in order),
            // so only the chunk gathers of the next set wait at a barrier
            stage_set();
            __syncthreads();
        }
    }
    if (norm_out) {
        __syncthreads();  // the tile-set's LDS is reused for the partial sums
        nrm = block_sum<NT>(nrm, reinterpret_cast<double *>(lds_raw));
        if (tid == 0) norm_out[blockIdx.x] = nrm;
    }
}

// ------------------------------------------------------------ relabelling

// LDS slot of group coordinate s: the low four bits XORed with a fold of the
// higher ones, so that sixteen lanes reading coordinates that differ in any
// four high bits mostly hit distinct banks.
__device__ __forceinline__ uint32_t perm_slot(uint32_t s) {
    return s ^ (((s >> 4) ^ (s >> 8)) & 15u);
}

// One relabelling pass: every group of 2^12 elements (fixed bits outside
// pos[]) is read with sixteen contiguous amplitudes per access, permuted
// through LDS and written back in place, again sixteen contiguous
// amplitudes per access.
template <typename T>
__global__ void __launch_bounds__(256) k_permute(Cx<T> *__restrict__ psi, PermArgs a) {
    static_assert(kPermBits == 12, "256 threads x 16 slots per group");
    __shared__ __align__(16) Cx<T> lds[1 << kPermBits];
    const uint32_t t = threadIdx.x;
    const uint64_t ngroups = 1ull << (a.n - kPermBits);
    uint32_t it = 0;    // D^-1 of the thread's bits of the output coordinate
    uint64_t toff = 0;  // the thread's bits (coordinates 0..7) as index bits
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if ((t >> j) & 1u) {
            it ^= a.inv[j];
            toff |= 1ull << a.pos[j];
        }
    }
    for (uint64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        uint64_t base = g;
#pragma unroll
        for (int j = 0; j < kPermBits; ++j) base = insert_zero64(base, a.pos[j]);
        base |= toff;
        Cx<T> r[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            uint64_t uo = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if ((u >> j) & 1) uo |= 1ull << a.pos[8 + j];
            r[u] = psi[base | uo];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) lds[perm_slot(t + 256u * (uint32_t)u)] = r[u];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 16; ++u) r[u] = lds[perm_slot(it ^ a.ioff[u])];
        __syncthreads();  // the group's LDS is reused by the next iteration
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            uint64_t uo = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if ((u >> j) & 1) uo |= 1ull << a.pos[8 + j];
            psi[base | uo] = r[u];
        }
    }
}

// ------------------------------------------------------------ reductions

// Neumaier-compensated accumulator.
struct Neu {
    double s = 0.0, c = 0.0;
    __device__ __forceinline__ void add(double v) {
        const double t = s + v;
        if (fabs(s) >= fabs(v))
            c += (s - t) + v;
        else
            c += (v - t) + s;
        s = t;
    }
    __device__ __forceinline__ double value() const { return s + c; }
};

// Fixed-shape tree over the block (deterministic for a fixed launch shape).
__device__ __forceinline__ double tree256(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < (unsigned)w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

template <typename T>
__global__ void __launch_bounds__(256) k_overlap(const Cx<T> *__restrict__ a,
                                                 const Cx<T> *__restrict__ b, uint64_t N,
                                                 double *__restrict__ part) {
    __shared__ double sh[256];
    Neu re, im;
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    for (uint64_t k = (uint64_t)blockIdx.x * 256u + threadIdx.x; k < N; k += stride) {
        const Cx<T> u = a[k], v = b[k];
        // conj(u) * v
        re.add((double)u.re * (double)v.re);
        re.add((double)u.im * (double)v.im);
        im.add((double)u.re * (double)v.im);
        im.add(-(double)u.im * (double)v.re);
    }
    const double r = tree256(re.value(), sh);
    const double i = tree256(im.value(), sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = r;
        part[2 * blockIdx.x + 1] = i;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_norm2(const Cx<T> *__restrict__ a, uint64_t N,
                                               double *__restrict__ part) {
    __shared__ double sh[256];
    Neu acc;
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    for (uint64_t k = (uint64_t)blockIdx.x * 256u + threadIdx.x; k < N; k += stride) {
        const Cx<T> u = a[k];
        acc.add((double)u.re * (double)u.re);
        acc.add((double)u.im * (double)u.im);
    }
    const double r = tree256(acc.value(), sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = r;
        part[2 * blockIdx.x + 1] = 0.0;
    }
}

// Sums `count` (re, im) partials into out[0..1] with one 256-thread block.
__global__ void __launch_bounds__(256) k_finish_pairs(const double *__restrict__ part,
                                                      unsigned count, double *__restrict__ out) {
    __shared__ double sh[256];
    Neu re, im;
    for (unsigned i = threadIdx.x; i < count; i += 256u) {
        re.add(part[2 * i]);
        im.add(part[2 * i + 1]);
    }
    const double r = tree256(re.value(), sh);
    const double m = tree256(im.value(), sh);
    if (threadIdx.x == 0) {
        out[0] = r;
        out[1] = m;
    }
}

// Norm hand-off, stage 1: block b sums its contiguous share of the
// `count` partials into stage[b] (fixed shape, deterministic).
__global__ void __launch_bounds__(256) k_renorm_stage1(const double *__restrict__ part,
                                                       unsigned count, double *__restrict__ stage) {
    __shared__ double sh[256];
    const unsigned per = (count + gridDim.x - 1) / gridDim.x;
    const unsigned lo = blockIdx.x * per;
    const unsigned hi = min(count, lo + per);
    Neu acc;
    for (unsigned i = lo + threadIdx.x; i < hi; i += 256u) acc.add(part[i]);
    const double s = tree256(acc.value(), sh);
    if (threadIdx.x == 0) stage[blockIdx.x] = s;
}

// Stage 2: sums the stage-1 values and writes 1/sqrt(sum).
__global__ void __launch_bounds__(256) k_renorm_finish(const double *__restrict__ stage,
                                                       unsigned count,
                                                       double *__restrict__ scale_out) {
    __shared__ double sh[256];
    Neu acc;
    for (unsigned i = threadIdx.x; i < count; i += 256u) acc.add(stage[i]);
    const double s = tree256(acc.value(), sh);
    if (threadIdx.x == 0) scale_out[0] = 1.0 / sqrt(s);
}

template <typename T>
__global__ void __launch_bounds__(256) k_scale(Cx<T> *__restrict__ a, uint64_t N,
                                               const double *__restrict__ scale) {
    const T s = (T)scale[0];
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    for (uint64_t k = (uint64_t)blockIdx.x * 256u + threadIdx.x; k < N; k += stride) {
        Cx<T> u = a[k];
        u.re *= s;
        u.im *= s;
        a[k] = u;
    }
}

// ------------------------------------------------------------- launchers

static unsigned ceil_div_u(uint64_t a, uint64_t b) { return (unsigned)((a + b - 1) / b); }
static unsigned capped_blocks(uint64_t want, unsigned cap) {
    const uint64_t c = std::max<uint64_t>(1, std::min<uint64_t>(cap, kMaxGridBlocks));
    return (unsigned)std::min<uint64_t>(want ? want : 1, c);
}

template <typename T>
static hipError_t plain_t(void *psi, const PlainArgs &a, hipStream_t s, unsigned cap) {
    constexpr int U = 4;
    if (a.x == 0) {
        const uint64_t N = 1ull << a.n;
        hipLaunchKernelGGL((k_plain_diag<T, U>), dim3(capped_blocks((N + 256u * U - 1) / (256u * U), cap)),
                           dim3(256), 0, s,
                           (Cx<T> *)psi, a, N);
    } else {
        const uint64_t np = 1ull << (a.n - 1);
        hipLaunchKernelGGL((k_plain_pair<T, U>), dim3(capped_blocks((np + 256u * U - 1) / (256u * U), cap)),
                           dim3(256), 0, s,
                           (Cx<T> *)psi, a, np);
    }
    return hipGetLastError();
}

hipError_t launch_plain(prx_dtype dt, void *psi, const PlainArgs &a, hipStream_t s, unsigned cap) {
    return dt == PRX_C64 ? plain_t<float>(psi, a, s, cap) : plain_t<double>(psi, a, s, cap);
}

unsigned permute_blocks(int n, unsigned cap) { return capped_blocks(1ull << (n - kPermBits), cap); }

hipError_t launch_permute(prx_dtype dt, void *psi, const PermArgs &a, hipStream_t s, unsigned cap) {
    const unsigned nb = permute_blocks(a.n, cap);
    if (dt == PRX_C64)
        hipLaunchKernelGGL(k_permute<float>, dim3(nb), dim3(256), 0, s, (Cx<float> *)psi, a);
    else
        hipLaunchKernelGGL(k_permute<double>, dim3(nb), dim3(256), 0, s, (Cx<double> *)psi, a);
    return hipGetLastError();
}

unsigned span_blocks(int n, int m, unsigned cap) {
    return capped_blocks(((1ull << (n - m)) + 255u) / 256u, cap);
}
unsigned tile_blocks(int n, int B, unsigned cap) { return capped_blocks(1ull << (n - B), cap); }
unsigned plain_blocks(int n, bool diag, unsigned cap) {
    const uint64_t items = diag ? (1ull << n) : (1ull << (n - 1));
    return capped_blocks((items + 1023u) / 1024u, cap);
}

// Persistent tile kernels stride over the 2^(n-B) tile-sets with the
// workgroups that fit on the device at once (cached per device and kernel).
static unsigned tile_grid(const void *kernel, int n, int B, int threads, unsigned cap) {
    struct Entry {
        const void *k;
        int dev;
        unsigned resident;
    };
    static Entry cache[64];
    static int used = 0;
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    int dev = 0;
    (void)hipGetDevice(&dev);
    unsigned resident = 0;
    for (int i = 0; i < used; ++i)
        if (cache[i].k == kernel && cache[i].dev == dev) resident = cache[i].resident;
    if (!resident) {
        int cus = 0, per = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess ||
            cus <= 0 || per <= 0)
            return tile_blocks(n, B, cap);  // one workgroup per tile-set
        resident = (unsigned)(cus * per);
        if (used < 64) cache[used++] = Entry{kernel, dev, resident};
    }
    const unsigned sets = tile_blocks(n, B, cap);
    return sets < resident ? sets : resident;
}

bool span_supported(prx_dtype, int m) { return m >= 1 && m <= 5; }

template <typename T>
static hipError_t span_t(int m, void *psi, const SpanArgs &a, const void *rots,
                         const double *rin, double *nout, hipStream_t s, unsigned *blocks,
                         unsigned cap) {
    const unsigned nb = span_blocks(a.n, m, cap);
    *blocks = nb;
    const RotRec<T> *r = (const RotRec<T> *)rots;
    Cx<T> *p = (Cx<T> *)psi;
    switch (m) {
    case 1: hipLaunchKernelGGL((k_span<T, 1>), dim3(nb), dim3(256), 0, s, p, a, r, rin, nout); break;
    case 2: hipLaunchKernelGGL((k_span<T, 2>), dim3(nb), dim3(256), 0, s, p, a, r, rin, nout); break;
    case 3: hipLaunchKernelGGL((k_span<T, 3>), dim3(nb), dim3(256), 0, s, p, a, r, rin, nout); break;
    case 4: hipLaunchKernelGGL((k_span<T, 4>), dim3(nb), dim3(256), 0, s, p, a, r, rin, nout); break;
    case 5: hipLaunchKernelGGL((k_span<T, 5>), dim3(nb), dim3(256), 0, s, p, a, r, rin, nout); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_span(prx_dtype dt, int m, void *psi, const SpanArgs &a, const void *rots,
                       const double *renorm_in, double *norm_out, hipStream_t s,
                       unsigned *blocks_out, unsigned cap) {
    return dt == PRX_C64 ? span_t<float>(m, psi, a, rots, renorm_in, norm_out, s, blocks_out, cap)
                         : span_t<double>(m, psi, a, rots, renorm_in, norm_out, s, blocks_out, cap);
}

// (B, M) pairs instantiated for the tile kernel.
#define PRX_TILE_SHAPES(X) X(10, 3) X(10, 4) X(11, 4) X(12, 4) X(12, 5) X(13, 4) X(13, 5) X(14, 4)

bool tile_supported(prx_dtype dt, int B, int m) {
// complex128 tile-sets up to 12 qubits, and 13 qubits (128 KiB) with rank-4
// chunks (rank 5 would need 256 registers per lane for the set and its
// prefetch)
#define PRX_TS(BB, MM) \
    if (B == BB && m == MM) return dt == PRX_C64 || BB <= 12 || (BB == 13 && MM == 4);
    PRX_TILE_SHAPES(PRX_TS)
#undef PRX_TS
    return false;
}

template <typename T, int B, int M>
static hipError_t tile_launch_one(void *psi, const TileArgs &a, const void *rots,
                                  const ChunkRec *chunks, const double *rin, double *nout,
                                  hipStream_t s, unsigned *blocks, unsigned cap) {
    const unsigned nb = TilePersist<T, B>::value
                            ? tile_grid((const void *)k_tile<T, B, M>, a.n, B, 1 << (B - M), cap)
                            : tile_blocks(a.n, B, cap);
    *blocks = nb;
    hipLaunchKernelGGL((k_tile<T, B, M>), dim3(nb), dim3(1 << (B - M)), 0, s, (Cx<T> *)psi, a,
                       (const RotRec<T> *)rots, chunks, rin, nout);
    return hipGetLastError();
}

template <typename T>
static hipError_t tile_t(int B, int m, void *psi, const TileArgs &a, const void *rots,
                         const ChunkRec *chunks, const double *rin, double *nout, hipStream_t s,
                         unsigned *blocks, unsigned cap) {
#define PRX_TL(BB, MM)                                                                         \
    if (B == BB && m == MM) {                                                                  \
        if constexpr (sizeof(T) == 4 || BB <= 12 || (BB == 13 && MM == 4))                    \
            return tile_launch_one<T, BB, MM>(psi, a, rots, chunks, rin, nout, s, blocks, cap); \
        return hipErrorInvalidValue;                                                      \
    }
    PRX_TILE_SHAPES(PRX_TL)
#undef PRX_TL
    return hipErrorInvalidValue;
}

hipError_t launch_tile(prx_dtype dt, int B, int m, void *psi, const TileArgs &a,
                       const void *rots, const ChunkRec *chunks, const double *renorm_in,
                       double *norm_out, hipStream_t s, unsigned *blocks_out, unsigned cap) {
    return dt == PRX_C64
               ? tile_t<float>(B, m, psi, a, rots, chunks, renorm_in, norm_out, s, blocks_out, cap)
               : tile_t<double>(B, m, psi, a, rots, chunks, renorm_in, norm_out, s, blocks_out, cap);
}

hipError_t launch_renorm_finish(const double *partials, unsigned count, double *scale_out,
                                hipStream_t s) {
    // scale_out[1 .. kRenormStage] holds the stage-1 sums
    double *stage = scale_out + 1;
    const unsigned g = count < 4096u ? 1u : kRenormStage;
    hipLaunchKernelGGL(k_renorm_stage1, dim3(g), dim3(256), 0, s, partials, count, stage);
    hipLaunchKernelGGL(k_renorm_finish, dim3(1), dim3(256), 0, s, stage, g, scale_out);
    return hipGetLastError();
}

static unsigned reduce_grid(uint64_t N) {
    const uint64_t want = (N + 256u * 8u - 1) / (256u * 8u);
    return (unsigned)(want < kReduceBlocks ? (want ? want : 1) : kReduceBlocks);
}

hipError_t launch_overlap(prx_dtype dt, const void *psi0, const void *psi, int n, double *ws,
                          hipStream_t s) {
    const uint64_t N = 1ull << n;
    const unsigned g = reduce_grid(N);
    if (dt == PRX_C64)
        hipLaunchKernelGGL(k_overlap<float>, dim3(g), dim3(256), 0, s, (const Cx<float> *)psi0,
                           (const Cx<float> *)psi, N, ws);
    else
        hipLaunchKernelGGL(k_overlap<double>, dim3(g), dim3(256), 0, s, (const Cx<double> *)psi0,
                           (const Cx<double> *)psi, N, ws);
    hipLaunchKernelGGL(k_finish_pairs, dim3(1), dim3(256), 0, s, ws, g, ws + 2 * kReduceBlocks);
    return hipGetLastError();
}

hipError_t launch_norm2(prx_dtype dt, const void *psi, int n, double *ws, hipStream_t s) {
    const uint64_t N = 1ull << n;
    const unsigned g = reduce_grid(N);
    if (dt == PRX_C64)
        hipLaunchKernelGGL(k_norm2<float>, dim3(g), dim3(256), 0, s, (const Cx<float> *)psi, N, ws);
    else
        hipLaunchKernelGGL(k_norm2<double>, dim3(g), dim3(256), 0, s, (const Cx<double> *)psi, N,
                           ws);
    hipLaunchKernelGGL(k_finish_pairs, dim3(1), dim3(256), 0, s, ws, g, ws + 2 * kReduceBlocks);
    return hipGetLastError();
}

hipError_t launch_scale(prx_dtype dt, void *psi, int n, const double *scale_dev,
                        hipStream_t s) {
    const uint64_t N = 1ull << n;
    const unsigned g = (unsigned)std::min<uint64_t>((N + 255) / 256, 256u * 64u);
    if (dt == PRX_C64)
        hipLaunchKernelGGL(k_scale<float>, dim3(g), dim3(256), 0, s, (Cx<float> *)psi, N, scale_dev);
    else
        hipLaunchKernelGGL(k_scale<double>, dim3(g), dim3(256), 0, s, (Cx<double> *)psi, N,
                           scale_dev);
    return hipGetLastError();
}

}  // namespace prx
