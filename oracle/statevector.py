"""FP64 state-vector oracle: Pauli action, rotation sequences, overlap, norm.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Definitions followed (paper, "Software implementation", "Mathematical model"
and Supplementary Methods, "Pauli-string bit representation"):
  * state: 2^n complex amplitudes, index k <-> basis state |k>;
  * P|i> = i^{popcount(x & z) mod 4} (-1)^{popcount(i & z)} |i XOR x>, the
    sign taken from the source index i;
  * exp(i phi P) = cos(phi) I + i sin(phi) P, applied as (i) the Pauli
    transform, then (ii) the linear combination;
  * overlap g = <psi0|psi> = sum_k conj(psi0[k]) psi[k] (Methods, "Data
    analysis", the signal g(t)).

Two implementations of the same definition: ``apply_rotations`` in numpy
(scatter written as an indexed assignment) and ``c_apply_rotations`` calling
the plain C loop in ``oracle.c``.  The tests check each against dense
matrices and against each other.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None


def _popcount(a: np.ndarray) -> np.ndarray:
    return np.bitwise_count(a)


def pauli_apply(x: int, z: int, psi: np.ndarray) -> np.ndarray:
    """Return P psi in the scatter form: w[i ^ x] = phase(i) psi[i]."""
    N = psi.shape[0]
    i = np.arange(N, dtype=np.uint64)
    x = np.uint64(x)
    z = np.uint64(z)
    yphase = (1, 1j, -1, -1j)[int(_popcount(np.array([x & z]))[0]) % 4]
    sign = 1.0 - 2.0 * (_popcount(i & z) & 1).astype(np.float64)
    w = np.zeros_like(psi)
    w[i ^ x] = yphase * sign * psi
    return w


def apply_rotations(psi0: np.ndarray, x, z, phi) -> np.ndarray:
    """psi_M = R_M ... R_1 psi0 with R_j = exp(i phi_j P_j); entry 0 first.

    FP64 throughout; cos and sin from the C library via numpy.
    """
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    for xj, zj, pj in zip(x, z, phi):
        w = pauli_apply(int(xj), int(zj), psi)
        psi = math.cos(float(pj)) * psi + 1j * math.sin(float(pj)) * w
    return psi


def overlap(psi0: np.ndarray, psi: np.ndarray) -> complex:
    """<psi0|psi>, each component summed with math.fsum (correctly rounded)."""
    p = np.conj(psi0) * psi
    return complex(math.fsum(p.real.tolist()), math.fsum(p.imag.tolist()))


def norm2(psi: np.ndarray) -> float:
    """sum_k |psi[k]|^2 with math.fsum."""
    return math.fsum((psi.real * psi.real).tolist() + (psi.imag * psi.imag).tolist())


# --------------------------------------------------------------------------
# C oracle (oracle.c), for sizes where numpy's temporaries are too slow.
# --------------------------------------------------------------------------

def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_apply.argtypes = [ctypes.c_int, ctypes.c_size_t, u64p, u64p, dp,
                                 ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_apply.restype = None
    lib.oracle_pauli_apply.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_pauli_apply.restype = None
    lib.oracle_overlap.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, dp]
    lib.oracle_overlap.restype = None
    lib.oracle_norm2.argtypes = [ctypes.c_int, ctypes.c_void_p]
    lib.oracle_norm2.restype = ctypes.c_double
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _nqubits(psi: np.ndarray) -> int:
    N = psi.shape[0]
    n = N.bit_length() - 1
    if N != 1 << n:
        raise ValueError("state length must be a power of two")
    return n


def c_apply_rotations(psi0: np.ndarray, x, z, phi, out: np.ndarray | None = None,
                      work: np.ndarray | None = None) -> np.ndarray:
    """Same as ``apply_rotations`` through the C loop (OpenMP over indices).

    ``out`` (complex128, may be psi0 itself) receives the result; ``work`` is
    optional scratch of the same length.
    """
    lib = _load()
    n = _nqubits(psi0)
    if out is None:
        out = np.array(psi0, dtype=np.complex128, copy=True)
    elif out is not psi0:
        out[:] = psi0
    assert out.dtype == np.complex128 and out.flags.c_contiguous
    if work is None:
        work = np.empty_like(out)
    x = np.ascontiguousarray(x, dtype=np.uint64)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_apply(n, len(x), x.ctypes.data_as(u64p), z.ctypes.data_as(u64p),
                     phi.ctypes.data_as(dp), out.ctypes.data, work.ctypes.data)
    return out


def c_pauli_apply(x: int, z: int, psi: np.ndarray) -> np.ndarray:
    lib = _load()
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    w = np.empty_like(psi)
    lib.oracle_pauli_apply(_nqubits(psi), int(x), int(z), psi.ctypes.data, w.ctypes.data)
    return w


def c_overlap(psi0: np.ndarray, psi: np.ndarray) -> complex:
    """<psi0|psi> with Neumaier-compensated FP64 sums (C loop, index order)."""
    lib = _load()
    a = np.ascontiguousarray(psi0, dtype=np.complex128)
    b = np.ascontiguousarray(psi, dtype=np.complex128)
    out = (ctypes.c_double * 2)()
    lib.oracle_overlap(_nqubits(a), a.ctypes.data, b.ctypes.data, out)
    return complex(out[0], out[1])


def c_norm2(psi: np.ndarray) -> float:
    lib = _load()
    a = np.ascontiguousarray(psi, dtype=np.complex128)
    return float(lib.oracle_norm2(_nqubits(a), a.ctypes.data))


def c_threads() -> int:
    return int(_load().oracle_threads())
