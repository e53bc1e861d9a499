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

// Flip the sign of v when bit 0 of p is set (an XOR on the sign bit).
__device__ __forceinline__ float flip(float v, uint32_t p) {
    return __uint_as_float(__float_as_uint(v) ^ (p << 31));
}
__device__ __forceinline__ double flip(double v, uint32_t p) {
    return __longlong_as_double(__double_as_longlong(v) ^ ((uint64_t)p << 63));
}

// ------------------------------------------------------ register updates
//
// amp[v], v in [0, 2^M), holds the amplitude at k0 XOR X(v), X(v) the XOR
// of the basis directions selected by v.  sigma(k0 XOR X(v)) =
// sigma0 XOR parity(v & zeta).  A rotation whose x is basis direction I
// pairs v with v | (1 << I).

template <typename T, int M, int I, bool IMAG>
__device__ __forceinline__ void rot_slot(Cx<T> (&amp)[1 << M], T g, uint32_t zeta) {
#pragma unroll
    for (int v = 0; v < (1 << M); ++v) {
        if (v & (1 << I)) continue;
        const int w = v | (1 << I);
        const T gw = flip(g, (uint32_t)__builtin_popcount((uint32_t)w & zeta) & 1u);
        const T gv = flip(g, (uint32_t)__builtin_popcount((uint32_t)v & zeta) & 1u);
        const Cx<T> av = amp[v], aw = amp[w];
        if (IMAG) {
            amp[v].re = fmat(-gw, aw.im, av.re);
            amp[v].im = fmat(gw, aw.re, av.im);
            amp[w].re = fmat(-gv, av.im, aw.re);
            amp[w].im = fmat(gv, av.re, aw.im);
        } else {
            amp[v].re = fmat(gw, aw.re, av.re);
            amp[v].im = fmat(gw, aw.im, av.im);
            amp[w].re = fmat(gv, av.re, aw.re);
            amp[w].im = fmat(gv, av.im, aw.im);
        }
    }
}

// x = 0: new = psi (1 + i tau' sigma), tau' = tan(phi) (tau is imaginary).
template <typename T, int M>
__device__ __forceinline__ void rot_diag(Cx<T> (&amp)[1 << M], T g, uint32_t zeta) {
#pragma unroll
    for (int v = 0; v < (1 << M); ++v) {
        const T gv = flip(g, (uint32_t)__builtin_popcount((uint32_t)v & zeta) & 1u);
        const Cx<T> av = amp[v];
        amp[v].re = fmat(-gv, av.im, av.re);
        amp[v].im = fmat(gv, av.re, av.im);
    }
}

template <typename T, int M, int I>
__device__ __forceinline__ void rot_slot_any(Cx<T> (&amp)[1 << M], T g, uint32_t zeta,
                                             bool imag) {
    if (imag)
        rot_slot<T, M, I, true>(amp, g, zeta);
    else
        rot_slot<T, M, I, false>(amp, g, zeta);
}

// Applies rotations [0, count) of `rots` to the thread's coset.
// k0: coset representative in the frame of rec.z; tsign_base: the tile
// index whose parity with rec.zhigh adds to the sign (0 for span passes).
template <typename T, int M>
__device__ __forceinline__ void apply_rots(Cx<T> (&amp)[1 << M], uint64_t k0, uint64_t tbase,
                                           const RotRec<T> *__restrict__ rots, uint32_t count) {
    for (uint32_t r = 0; r < count; ++r) {
        const RotRec<T> rec = rots[r];
        const uint32_t s0 = parity64(k0 & rec.z) ^ parity64(tbase & rec.zhigh);
        const T g = pin(flip(rec.tau, s0));
        const uint32_t slot = rec.info & 15u;
        const bool imag = (rec.info >> 4) & 1u;
        const uint32_t zeta = (rec.info >> 8) & 0xffu;
        // one uniform branch per slot, each updating amp in place
        if (slot == 0) rot_slot_any<T, M, 0>(amp, g, zeta, imag);
        if constexpr (M > 1) if (slot == 1) rot_slot_any<T, M, 1>(amp, g, zeta, imag);
        if constexpr (M > 2) if (slot == 2) rot_slot_any<T, M, 2>(amp, g, zeta, imag);
        if constexpr (M > 3) if (slot == 3) rot_slot_any<T, M, 3>(amp, g, zeta, imag);
        if constexpr (M > 4) if (slot == 4) rot_slot_any<T, M, 4>(amp, g, zeta, imag);
        if constexpr (M > 5) if (slot == 5) rot_slot_any<T, M, 5>(amp, g, zeta, imag);
        if (slot == kSlotDiag) rot_diag<T, M>(amp, g, zeta);
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
