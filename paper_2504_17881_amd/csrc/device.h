// Device routines shared by the sweep kernels (kernels.hip) and the
// batched persistent kernel (batch.hip): index arithmetic, sign flips and
// the in-register rotation updates of a coset.
#pragma once

#include "internal.h"

namespace prx {

template <typename T>
struct Cx {
    T re, im;
};

__device__ __forceinline__ uint64_t insert_zero64(uint64_t v, uint32_t p) {
    const uint64_t lo = v & ((1ull << p) - 1ull);
    return ((v >> p) << (p + 1)) | lo;
}
__device__ __forceinline__ uint32_t insert_zero32(uint32_t v, uint32_t p) {
    const uint32_t lo = v & ((1u << p) - 1u);
    return ((v >> p) << (p + 1)) | lo;
}
__device__ __forceinline__ uint32_t parity64(uint64_t v) { return __popcll(v) & 1u; }

__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Keeps a value materialised in a register, so that later sign flips of it
// are single XORs instead of being re-derived from their inputs.
__device__ __forceinline__ float pin(float v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ double pin(double v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ uint32_t pin(uint32_t v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Flip the sign of v when bit 0 of p is set (an XOR on the sign bit).
__device__ __forceinline__ float flip(float v, uint32_t p) {
    return __uint_as_float(__float_as_uint(v) ^ (p << 31));
}
__device__ __forceinline__ double flip(double v, uint32_t p) {
    return __longlong_as_double(__double_as_longlong(v) ^ ((uint64_t)p << 63));
}
// The same for any count p: adding (p << 31) to the bit pattern flips the
// sign bit exactly when p is odd (the carry out of bit 31 is dropped), which
// is one shift-add instruction.
__device__ __forceinline__ float flip_add(float v, uint32_t p) {
    return __uint_as_float(__float_as_uint(v) + (p << 31));
}
__device__ __forceinline__ double flip_add(double v, uint32_t p) {
    const uint64_t u = __double_as_longlong(v);
    const uint32_t hi = (uint32_t)(u >> 32) + (p << 31);
    return __longlong_as_double((u & 0xffffffffull) | ((uint64_t)hi << 32));
}

// ------------------------------------------------------ register updates
//
// amp[v], v in [0, 2^M), holds the amplitude at k0 XOR X(v), X(v) the XOR
// of the basis directions selected by v.  sigma(k0 XOR X(v)) =
// sigma0 XOR parity(v & zeta).  A rotation whose x is basis direction I
// pairs v with v | (1 << I).

// In-place update of one pair (a, b) (see RotRec):
//     a <- a + ga * b,   then  b <- b + gb * a       (real tau)
//     a <- a + i ga * b, then  b <- b + i gb * a     (imaginary tau)
// Tied asm operands keep a and b in their registers, so the rotation loop
// needs no register copies whichever slot it takes.
__device__ __forceinline__ void pair_real(Cx<float> &a, Cx<float> &b, float ga, float gb) {
    asm("v_fma_f32 %0, %4, %2, %0\n\t"
        "v_fma_f32 %1, %4, %3, %1\n\t"
        "v_fma_f32 %2, %5, %0, %2\n\t"
        "v_fma_f32 %3, %5, %1, %3"
        : "+v"(a.re), "+v"(a.im), "+v"(b.re), "+v"(b.im)
        : "v"(ga), "v"(gb));
}
__device__ __forceinline__ void pair_imag(Cx<float> &a, Cx<float> &b, float ga, float gb) {
    asm("v_fma_f32 %0, -%4, %3, %0\n\t"
        "v_fma_f32 %1, %4, %2, %1\n\t"
        "v_fma_f32 %2, -%5, %1, %2\n\t"
        "v_fma_f32 %3, %5, %0, %3"
        : "+v"(a.re), "+v"(a.im), "+v"(b.re), "+v"(b.im)
        : "v"(ga), "v"(gb));
}
// a <- a (1 + i g)
__device__ __forceinline__ void self_imag(Cx<float> &a, float g) {
    float t;
    asm("v_mov_b32 %2, %0\n\t"
        "v_fma_f32 %0, -%3, %1, %0\n\t"
        "v_fma_f32 %1, %3, %2, %1"
        : "+v"(a.re), "+v"(a.im), "=&v"(t)
        : "v"(g));
}
__device__ __forceinline__ void pair_real(Cx<double> &a, Cx<double> &b, double ga, double gb) {
    asm("v_fma_f64 %0, %4, %2, %0\n\t"
        "v_fma_f64 %1, %4, %3, %1\n\t"
        "v_fma_f64 %2, %5, %0, %2\n\t"
        "v_fma_f64 %3, %5, %1, %3"
        : "+v"(a.re), "+v"(a.im), "+v"(b.re), "+v"(b.im)
        : "v"(ga), "v"(gb));
}
__device__ __forceinline__ void pair_imag(Cx<double> &a, Cx<double> &b, double ga, double gb) {
    asm("v_fma_f64 %0, -%4, %3, %0\n\t"
        "v_fma_f64 %1, %4, %2, %1\n\t"
        "v_fma_f64 %2, -%5, %1, %2\n\t"
        "v_fma_f64 %3, %5, %0, %3"
        : "+v"(a.re), "+v"(a.im), "+v"(b.re), "+v"(b.im)
        : "v"(ga), "v"(gb));
}
__device__ __forceinline__ void self_imag(Cx<double> &a, double g) {
    double t;
    asm("v_mov_b64 %2, %0\n\t"
        "v_fma_f64 %0, -%3, %1, %0\n\t"
        "v_fma_f64 %1, %3, %2, %1"
        : "+v"(a.re), "+v"(a.im), "=&v"(t)
        : "v"(g));
}

// The same pair update with both coefficients negated when NEG, through the
// FMA's source negation modifiers (no extra instruction).
template <bool IMAG, bool NEG>
__device__ __forceinline__ void pair_s(Cx<float> &a, Cx<float> &b, float ga, float gb) {
    if constexpr (!IMAG && !NEG) {
        pair_real(a, b, ga, gb);
    } else if constexpr (!IMAG && NEG) {
        asm("v_fma_f32 %0, -%4, %2, %0\n\t"
            "v_fma_f32 %1, -%4, %3, %1\n\t"
            "v_fma_f32 %2, -%5, %0, %2\n\t"
            "v_fma_f32 %3, -%5, %1, %3"
            : "+v"(a.re), "+v"(a.im), "+v"(b.re), "+v"(b.im)
            : "v"(ga), "v"(gb));
    } else if constexpr (IMAG && !NEG) {
        pair_imag(a, b, ga, gb);
    } else {
        asm("v_fma_f32 %0, %4, %3, %0\n\t"
            "v_fma_f32 %1, -%4, %2, %1\n\t"
            "v_fma_f32 %2, %5, %1, %2\n\t"
            "v_fma_f32 %3, -%5, %0, %3"
            : "+v"(a.re), "+v"(a.im), "+v"(b.re), "+v"(b.im)
            : "v"(ga), "v"(gb));
    }
}
template <bool IMAG, bool NEG>
__device__ __forceinline__ void pair_s(Cx<double> &a, Cx<double> &b, double ga, double gb) {
    if constexpr (!IMAG && !NEG) {
        pair_real(a, b, ga, gb);
    } else if constexpr (!IMAG && NEG) {
        asm("v_fma_f64 %0, -%4, %2, %0\n\t"
            "v_fma_f64 %1, -%4, %3, %1\n\t"
            "v_fma_f64 %2, -%5, %0, %2\n\t"
            "v_fma_f64 %3, -%5, %1, %3"
            : "+v"(a.re), "+v"(a.im), "+v"(b.re), "+v"(b.im)
            : "v"(ga), "v"(gb));
    } else if constexpr (IMAG && !NEG) {
        pair_imag(a, b, ga, gb);
    } else {
        asm("v_fma_f64 %0, %4, %3, %0\n\t"
            "v_fma_f64 %1, -%4, %2, %1\n\t"
            "v_fma_f64 %2, %5, %1, %2\n\t"
            "v_fma_f64 %3, -%5, %0, %3"
            : "+v"(a.re), "+v"(a.im), "+v"(b.re), "+v"(b.im)
            : "v"(ga), "v"(gb));
    }
}

// Sign masks S[v] = parity(v & zeta) << 31 for all coset labels v, built
// incrementally (one XOR per label).
template <int M>
__device__ __forceinline__ void sign_masks(uint32_t (&S)[1 << M], uint32_t zeta) {
    S[0] = 0;
#pragma unroll
    for (int v = 1; v < (1 << M); ++v)
        S[v] = S[v & (v - 1)] ^ (((zeta >> __builtin_ctz(v)) & 1u) << 31);
}

__device__ __forceinline__ float flipm(float v, uint32_t m) { return __uint_as_float(__float_as_uint(v) ^ m); }
__device__ __forceinline__ double flipm(double v, uint32_t m) {
    return __longlong_as_double(__double_as_longlong(v) ^ ((uint64_t)m << 32));
}

template <typename T, int M, int I, bool IMAG>
__device__ __forceinline__ void rot_slot(Cx<T> (&amp)[1 << M], T ga, T gb, uint32_t zeta) {
    uint32_t S[1 << M];
    sign_masks<M>(S, zeta);
#pragma unroll
    for (int v = 0; v < (1 << M); ++v) {
        if (v & (1 << I)) continue;
        const int w = v | (1 << I);
        if (IMAG)
            pair_imag(amp[v], amp[w], flipm(ga, S[w]), flipm(gb, S[v]));
        else
            pair_real(amp[v], amp[w], flipm(ga, S[w]), flipm(gb, S[v]));
    }
}

// Static-sign form for ranks up to kStaticSignRank.  Pair (v, w = v | 2^I)
// takes ga s_w and gb s_v, s_u = s0 (-1)^parity(u & zeta).  With ga
// pre-multiplied by (-1)^zeta_I (a uniform flip), both become s0 times
// (-1)^parity(c(v) & zp), c(v) being v with bit I removed and zp zeta with
// bit I removed: for each of the 2^(M-1) values of zp the signs are
// compile-time constants and go into negation modifiers.
__host__ __device__ constexpr int drop_bit(int v, int I) {
    return ((v >> (I + 1)) << I) | (v & ((1 << I) - 1));
}

template <typename T, int M, int I, bool IMAG, int ZP, int V = 0>
__device__ __forceinline__ void rot_fixed(Cx<T> (&amp)[1 << M], T ga, T gb) {
    if constexpr (V < (1 << M)) {
        if constexpr (!(V & (1 << I))) {
            constexpr bool neg = (__builtin_popcount(drop_bit(V, I) & ZP) & 1) != 0;
            pair_s<IMAG, neg>(amp[V], amp[V | (1 << I)], ga, gb);
        }
        rot_fixed<T, M, I, IMAG, ZP, V + 1>(amp, ga, gb);
    }
}

// x = 0: new = psi (1 + i tan(phi) sigma) (tau is imaginary).
template <typename T, int M>
__device__ __forceinline__ void rot_diag(Cx<T> (&amp)[1 << M], T g, uint32_t zeta) {
    uint32_t S[1 << M];
    sign_masks<M>(S, zeta);
#pragma unroll
    for (int v = 0; v < (1 << M); ++v) self_imag(amp[v], flipm(g, S[v]));
}

// Element v's pending factor: the product of K over the slots set in v.
template <int M>
__device__ __forceinline__ void pending_factors(double (&F)[1 << M], const double *K) {
    F[0] = 1.0;
#pragma unroll
    for (int v = 1; v < (1 << M); ++v) F[v] = F[v & (v - 1)] * K[__builtin_ctz(v)];
}

template <typename T, int M, int I>
__device__ __forceinline__ void rot_slot_any(Cx<T> (&amp)[1 << M], T ga, T gb, uint32_t zeta,
                                             bool imag) {
    if (imag)
        rot_slot<T, M, I, true>(amp, ga, gb, zeta);
    else
        rot_slot<T, M, I, false>(amp, ga, gb, zeta);
}

// The complex64 rank-4 variants as one jump table (rot_jump_f32m4.inc,
// written by gen_rot_jump.py): a computed jump to variant var (< 64) of
// equal-sized blocks instead of a 7-level branch tree.  var is uniform (one
// rotation record per wave); the table clamps it to 63.
#include "rot_jump_f32m4.inc"
__device__ __forceinline__ void rot_jump(Cx<float> (&amp)[16], float ga, float gb, uint32_t var) {
    uint32_t t;
    asm(PRX_ROT_JUMP_F32M4
        : "+v"(amp[0].re), "+v"(amp[0].im), "+v"(amp[1].re), "+v"(amp[1].im),
          "+v"(amp[2].re), "+v"(amp[2].im), "+v"(amp[3].re), "+v"(amp[3].im),
          "+v"(amp[4].re), "+v"(amp[4].im), "+v"(amp[5].re), "+v"(amp[5].im),
          "+v"(amp[6].re), "+v"(amp[6].im), "+v"(amp[7].re), "+v"(amp[7].im),
          "+v"(amp[8].re), "+v"(amp[8].im), "+v"(amp[9].re), "+v"(amp[9].im),
          "+v"(amp[10].re), "+v"(amp[10].im), "+v"(amp[11].re), "+v"(amp[11].im),
          "+v"(amp[12].re), "+v"(amp[12].im), "+v"(amp[13].re), "+v"(amp[13].im),
          "+v"(amp[14].re), "+v"(amp[14].im), "+v"(amp[15].re), "+v"(amp[15].im),
          "=&s"(t)
        : "v"(ga), "v"(gb), "s"(__builtin_amdgcn_readfirstlane(var))
        : "s90", "s91", "scc");
}

// The complex128 variants as the same kind of table (rot_jump_f64m4.inc).
#include "rot_jump_f64m4.inc"
__device__ __forceinline__ void rot_jump(Cx<double> (&amp)[16], double ga, double gb,
                                         uint32_t var) {
    uint32_t t;
    asm(PRX_ROT_JUMP_F64M4
        : "+v"(amp[0].re), "+v"(amp[0].im), "+v"(amp[1].re), "+v"(amp[1].im),
          "+v"(amp[2].re), "+v"(amp[2].im), "+v"(amp[3].re), "+v"(amp[3].im),
          "+v"(amp[4].re), "+v"(amp[4].im), "+v"(amp[5].re), "+v"(amp[5].im),
          "+v"(amp[6].re), "+v"(amp[6].im), "+v"(amp[7].re), "+v"(amp[7].im),
          "+v"(amp[8].re), "+v"(amp[8].im), "+v"(amp[9].re), "+v"(amp[9].im),
          "+v"(amp[10].re), "+v"(amp[10].im), "+v"(amp[11].re), "+v"(amp[11].im),
          "+v"(amp[12].re), "+v"(amp[12].im), "+v"(amp[13].re), "+v"(amp[13].im),
          "+v"(amp[14].re), "+v"(amp[14].im), "+v"(amp[15].re), "+v"(amp[15].im),
          "=&s"(t)
        : "v"(ga), "v"(gb), "s"(__builtin_amdgcn_readfirstlane(var))
        : "s90", "s91", "scc");
}

// Binary dispatch of a static-sign rotation on the uniform variant index
// var = slot 2^M + imag 2^(M-1) + zp in [LO, HI); var = M 2^M is the
// diagonal (x = 0) rotation.
template <typename T, int M, int LO, int HI>
__device__ __forceinline__ void rot_var(Cx<T> (&amp)[1 << M], T ga, T gb, uint32_t var,
                                        uint32_t zeta) {
    if constexpr (HI - LO == 1) {
        if constexpr (LO == (M << M)) {
            rot_diag<T, M>(amp, ga, zeta);
        } else {
            constexpr int I = LO >> M;
            constexpr bool IMAG = ((LO >> (M - 1)) & 1) != 0;
            constexpr int ZP = LO & ((1 << (M - 1)) - 1);
            rot_fixed<T, M, I, IMAG, ZP>(amp, ga, gb);
        }
    } else {
        constexpr int MID = (LO + HI) / 2;
        if (var < (uint32_t)MID)
            rot_var<T, M, LO, MID>(amp, ga, gb, var, zeta);
        else
            rot_var<T, M, MID, HI>(amp, ga, gb, var, zeta);
    }
}

// The same variants as threaded code (rot_loop_f32m4.inc): runs the records
// at plo:phi until cnt reaches zero or a diagonal record comes up (left
// unconsumed); k0 is the lane's coset representative, tb the base tile
// index.  The pointer and count are uniform; so are their new values.  It
// loads the record after the current one early, so every rotation table is
// followed by kRecordReadAhead readable bytes (plan and batch workspaces).
#include "rot_loop_f32m4.inc"
__device__ __forceinline__ void rot_loop(Cx<float> (&amp)[16], uint32_t k0, uint64_t tb,
                                         uint32_t &plo, uint32_t &phi, uint32_t &cnt) {
    uint32_t ga, gb;
    asm volatile(PRX_ROT_LOOP_F32M4
        : "+v"(amp[0].re), "+v"(amp[0].im), "+v"(amp[1].re), "+v"(amp[1].im),
          "+v"(amp[2].re), "+v"(amp[2].im), "+v"(amp[3].re), "+v"(amp[3].im),
          "+v"(amp[4].re), "+v"(amp[4].im), "+v"(amp[5].re), "+v"(amp[5].im),
          "+v"(amp[6].re), "+v"(amp[6].im), "+v"(amp[7].re), "+v"(amp[7].im),
          "+v"(amp[8].re), "+v"(amp[8].im), "+v"(amp[9].re), "+v"(amp[9].im),
          "+v"(amp[10].re), "+v"(amp[10].im), "+v"(amp[11].re), "+v"(amp[11].im),
          "+v"(amp[12].re), "+v"(amp[12].im), "+v"(amp[13].re), "+v"(amp[13].im),
          "+v"(amp[14].re), "+v"(amp[14].im), "+v"(amp[15].re), "+v"(amp[15].im),
          [plo] "+s"(plo), [phi] "+s"(phi), [cnt] "+s"(cnt), [ga] "=&v"(ga), [gb] "=&v"(gb)
        : [k0] "v"(k0), [tb] "s"(tb)
        : "s76", "s77", "s78", "s79", "s80", "s81", "s82", "s83", "s84", "s85", "s86", "s87",
          "s88", "s89", "s90", "s91", "scc", "memory");
    plo = __builtin_amdgcn_readfirstlane(plo);
    phi = __builtin_amdgcn_readfirstlane(phi);
    cnt = __builtin_amdgcn_readfirstlane(cnt);
}

// The complex128 form (rot_loop_f64m4.inc): 40-byte records, the lane sign
// applied as a factor of +-1.0; same contract.
#include "rot_loop_f64m4.inc"
__device__ __forceinline__ void rot_loop(Cx<double> (&amp)[16], uint32_t k0, uint64_t tb,
                                         uint32_t &plo, uint32_t &phi, uint32_t &cnt) {
    double ga, gb, sg;
    uint32_t t;
    asm volatile(PRX_ROT_LOOP_F64M4
        : "+v"(amp[0].re), "+v"(amp[0].im), "+v"(amp[1].re), "+v"(amp[1].im),
          "+v"(amp[2].re), "+v"(amp[2].im), "+v"(amp[3].re), "+v"(amp[3].im),
          "+v"(amp[4].re), "+v"(amp[4].im), "+v"(amp[5].re), "+v"(amp[5].im),
          "+v"(amp[6].re), "+v"(amp[6].im), "+v"(amp[7].re), "+v"(amp[7].im),
          "+v"(amp[8].re), "+v"(amp[8].im), "+v"(amp[9].re), "+v"(amp[9].im),
          "+v"(amp[10].re), "+v"(amp[10].im), "+v"(amp[11].re), "+v"(amp[11].im),
          "+v"(amp[12].re), "+v"(amp[12].im), "+v"(amp[13].re), "+v"(amp[13].im),
          "+v"(amp[14].re), "+v"(amp[14].im), "+v"(amp[15].re), "+v"(amp[15].im),
          [plo] "+s"(plo), [phi] "+s"(phi), [cnt] "+s"(cnt), [ga] "=&v"(ga), [gb] "=&v"(gb),
          [sg] "=&v"(sg), [t] "=&v"(t)
        : [k0] "v"(k0), [tb] "s"(tb)
        : "s76", "s77", "s78", "s79", "s80", "s81", "s82", "s83", "s84", "s85", "s86", "s87",
          "s88", "s89", "s90", "s91", "s92", "s93", "scc", "memory");
    plo = __builtin_amdgcn_readfirstlane(plo);
    phi = __builtin_amdgcn_readfirstlane(phi);
    cnt = __builtin_amdgcn_readfirstlane(cnt);
}

// Applies rotations [0, count) of `rots` to the thread's coset.
// k0: coset representative in the frame of rec.z (32-bit in a tile frame);
// tbase: the tile index whose parity with rec.zhigh adds to the sign (0 for
// span passes).
template <typename T, int M, typename K0>
__device__ __forceinline__ void apply_rots(Cx<T> (&amp)[1 << M], K0 k0, uint64_t tbase,
                                           const RotRec<T> *__restrict__ rots, uint32_t count) {
    if constexpr (M == 4 && sizeof(K0) == 4) {
        // rank-4 tile chunks: the threaded loop, stopping for the diagonal
        // records, which take the compiled path below
        const uint64_t p0 = (uint64_t)rots;
        uint32_t plo = __builtin_amdgcn_readfirstlane((uint32_t)p0);
        uint32_t phi = __builtin_amdgcn_readfirstlane((uint32_t)(p0 >> 32));
        uint32_t cnt = __builtin_amdgcn_readfirstlane(count);
        while (true) {
            rot_loop(amp, k0, tbase, plo, phi, cnt);
            if (cnt == 0u) break;
            // the record's fields through the constant address space (scalar
            // loads: the pointer is uniform)
            typedef const __attribute__((address_space(4))) RotRec<T> *ConstRec;
            const ConstRec rp = (ConstRec)((((uint64_t)phi) << 32) | plo);
            const uint64_t rz = rp->z, rzhigh = rp->zhigh;
            const uint32_t info = rp->info;
            const T tau_a = rp->tau_a;
            const uint32_t zeta = (info >> 8) & 0xffu;
            const uint32_t tpar =
                __builtin_amdgcn_readfirstlane((uint32_t)__builtin_popcountll(tbase & rzhigh));
            uint32_t c;
            asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(c) : "v"(k0 & (uint32_t)rz), "s"(tpar));
            if constexpr (sizeof(T) == 4) {
                uint32_t ua;
                asm("v_lshl_add_u32 %0, %1, 31, %2"
                    : "=v"(ua)
                    : "v"(c), "s"(__builtin_amdgcn_readfirstlane(__float_as_uint(tau_a))));
                rot_diag<T, M>(amp, __uint_as_float(ua), zeta);
            } else {
                rot_diag<T, M>(amp, pin(flip_add(tau_a, c)), zeta);
            }
            const uint64_t pn = (((uint64_t)phi << 32) | plo) + sizeof(RotRec<T>);
            plo = (uint32_t)pn;
            phi = (uint32_t)(pn >> 32);
            cnt -= 1u;
        }
        return;
    }
    for (uint32_t r = 0; r < count; ++r) {
        const RotRec<T> rec = rots[r];
        const uint32_t slot = rec.info & 15u;
        const bool imag = (rec.info >> 4) & 1u;
        const uint32_t zeta = (rec.info >> 8) & 0xffu;
        // uniform part of the sign, then one AND and one count per lane
        const uint32_t tpar = (uint32_t)__builtin_popcountll(tbase & rec.zhigh);
        uint32_t cnt;  // parity in bit 0
        if constexpr (sizeof(K0) == 4) {
            // one AND and one count that adds the uniform part
            const uint32_t m = k0 & (uint32_t)rec.z;
            asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(cnt) : "v"(m), "s"(tpar));
        } else {
            cnt = (uint32_t)__builtin_popcountll(k0 & rec.z) + tpar;
        }
        const uint32_t s0 = cnt & 1u;
        if constexpr (M <= kStaticSignRank) {
            // tau_a arrives multiplied by (-1)^zeta_slot: both pair
            // coefficients then share the pattern (-1)^parity(c(v) & zp)
            T ga, gb;
            if constexpr (sizeof(T) == 4) {
                // one shift-add per coefficient (see flip_add)
                uint32_t ua, ub;
                asm("v_lshl_add_u32 %0, %1, 31, %2" : "=v"(ua) : "v"(cnt), "s"(__float_as_uint(rec.tau_a)));
                asm("v_lshl_add_u32 %0, %1, 31, %2" : "=v"(ub) : "v"(cnt), "s"(__float_as_uint(rec.tau_b)));
                ga = __uint_as_float(ua);
                gb = __uint_as_float(ub);
            } else {
                ga = pin(flip_add(rec.tau_a, cnt));
                gb = pin(flip_add(rec.tau_b, cnt));
            }
            const uint32_t var = (rec.info >> 16) & 0xffu;
            if constexpr (M == 4) {
                if (var == (uint32_t)(M << M))
                    rot_diag<T, M>(amp, ga, zeta);
                else
                    rot_jump(amp, ga, gb, var);
            } else {
                rot_var<T, M, 0, (M << M) + 1>(amp, ga, gb, var, zeta);
            }
            continue;
        }
        const T ga = pin(flip(rec.tau_a, s0));
        const T gb = pin(flip(rec.tau_b, s0));
        // one uniform branch per slot, each updating amp in place
        if (slot == 0) rot_slot_any<T, M, 0>(amp, ga, gb, zeta, imag);
        if constexpr (M > 1) if (slot == 1) rot_slot_any<T, M, 1>(amp, ga, gb, zeta, imag);
        if constexpr (M > 2) if (slot == 2) rot_slot_any<T, M, 2>(amp, ga, gb, zeta, imag);
        if constexpr (M > 3) if (slot == 3) rot_slot_any<T, M, 3>(amp, ga, gb, zeta, imag);
        if constexpr (M > 4) if (slot == 4) rot_slot_any<T, M, 4>(amp, ga, gb, zeta, imag);
        if constexpr (M > 5) if (slot == 5) rot_slot_any<T, M, 5>(amp, ga, gb, zeta, imag);
        if (slot == kSlotDiag) rot_diag<T, M>(amp, ga, zeta);
    }
}

// ------------------------------------------------------------ tile chunks
//
// A tile-set of 2^B amplitudes sits in LDS (byte offsets from lds_raw).  For
// each chunk, thread tid gathers the coset k0(tid) XOR span(basis) into
// registers (k0(tid) = XOR of the chunk's complement vectors over the bits
// of tid), applies the chunk's rotations, multiplies by the pending factors
// of the coset labels and scatters back; a barrier separates chunks.

// a ^ (m & c) in one gfx950 three-input bit operation (truth table 0x78
// over the inputs a, m, c taken as bits 2, 1, 0 of the table index); the
// compiler emits an AND and an XOR for the chunk representative otherwise.
__device__ __forceinline__ uint32_t xor_and(uint32_t a, uint32_t m, uint32_t c) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x78" : "=v"(r) : "v"(a), "v"(m), "s"(c));
    return r;
}

// All-ones masks of the thread index bits: a chunk's representative is then
// one AND-XOR per bit (pinned in registers).
template <int NB>
__device__ __forceinline__ void tile_thread_masks(uint32_t tid, uint32_t (&tmask)[NB]) {
#pragma unroll
    for (int i = 0; i < NB; ++i) tmask[i] = pin(0u - ((tid >> i) & 1u));
}

template <typename T, int B, int M>
__device__ __forceinline__ void tile_chunks(unsigned char *lds_raw, const uint32_t (&tmask)[B - M],
                                            uint64_t tb, const ChunkRec *__restrict__ chunks,
                                            uint32_t count, const RotRec<T> *__restrict__ rots) {
    // LDS byte offsets: the XOR of indices commutes with the element shift
    constexpr uint32_t SH = sizeof(Cx<T>) == 8 ? 3u : 4u;
    for (uint32_t c = 0; c < count; ++c) {
        const ChunkRec ch = chunks[c];
        uint32_t k0 = 0;
#pragma unroll
        for (int i = 0; i < B - M; ++i) k0 = xor_and(k0, tmask[i], (uint32_t)ch.cvec[i]);
        const uint32_t k0b = k0 << SH;
        uint32_t Xb[1 << M];
        Xb[0] = 0;
#pragma unroll
        for (int v = 1; v < (1 << M); ++v)
            Xb[v] = Xb[v & (v - 1)] ^ (ch.basis[__builtin_ctz(v)] << SH);
        Cx<T> amp[1 << M];
#pragma unroll
        for (int v = 0; v < (1 << M); ++v)
            amp[v] = *reinterpret_cast<const Cx<T> *>(lds_raw + (k0b ^ Xb[v]));
        apply_rots<T, M>(amp, k0, tb, rots + ch.rot_begin, ch.rot_count);
#pragma unroll
        for (int v = 0; v < (1 << M); ++v) {
            T f;
            if constexpr (sizeof(T) == 4)
                f = ch.facf[v];
            else
                f = ch.facd[v];
            Cx<T> o;
            o.re = amp[v].re * f;
            o.im = amp[v].im * f;
            *reinterpret_cast<Cx<T> *>(lds_raw + (k0b ^ Xb[v])) = o;
        }
        __syncthreads();
    }
}

// FP64 block sum of one value per thread; result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if constexpr (NT > 64) {
        if (lane == 0) red[wave] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int i = 0; i < NT / 64; ++i) s += red[i];
            v = s;
        }
    }
    return v;
}

}  // namespace prx
