"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only *draws* inputs: states, Pauli masks, coefficients, qubit
counts.  It holds none of the method's arithmetic (no Pauli action, no
rotation, no schedule, no overlap), so that the oracle and the HIP path can
both take their inputs from here without sharing any computation.

Pauli strings are handed out in the two-mask form used throughout the
package: bit q of ``x`` is set when the letter on qubit q is X or Y, bit q of
``z`` is set when it is Y or Z (Supplementary Methods, "Pauli-string bit
representation").  Qubit 0 is the least significant bit of an amplitude index
("Software implementation": qubits run from least to most significant).

The paper's workload is a Jordan-Wigner-mapped electronic-structure
Hamiltonian of a ruthenium complex (Methods, "Hamiltonian preparation"), whose
data is not available here.  ``jw_hamiltonian`` stands in for it with the same
shape: terms are Z-strings between X/Y endpoints (one segment, as in a hopping
term, or two disjoint segments, as in a double excitation), weights skewed so
that 60% of terms have weight at most 4, signed log-normal magnitudes.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gaussian_state",
    "basis_index",
    "random_pauli_rotations",
    "jw_hamiltonian",
    "batch_qubit_counts",
    "WORKLOADS",
]


def gaussian_state(n: int, seed: int = 0) -> np.ndarray:
    """i.i.d. standard complex Gaussian amplitudes, normalised in FP64.

    All real parts are drawn first, then all imaginary parts, from
    ``numpy.random.default_rng(seed)``.  Returns complex128 of length 2**n.
    """
    rng = np.random.default_rng(seed)
    N = 1 << n
    re = rng.standard_normal(N)
    im = rng.standard_normal(N)
    psi = re + 1j * im
    psi /= np.sqrt(np.sum(re * re) + np.sum(im * im))
    return psi.astype(np.complex128)


def basis_index(n: int) -> int:
    """Index of the basis state with the low floor(n/2) bits set."""
    return (1 << (n // 2)) - 1


def random_pauli_rotations(n: int, M: int, seed: int = 1):
    """M uniformly random non-identity Pauli strings on n qubits with angles
    uniform in [-pi, pi].

    A letter uniform over {I, X, Y, Z} on every qubit is the same as two
    independent uniform n-bit masks (x, z); the all-zero pair (the identity)
    is redrawn.  Returns (x uint64[M], z uint64[M], phi float64[M]).
    """
    rng = np.random.default_rng(seed)
    hi = 1 << n
    x = np.empty(M, dtype=np.uint64)
    z = np.empty(M, dtype=np.uint64)
    phi = np.empty(M, dtype=np.float64)
    for j in range(M):
        while True:
            xv = int(rng.integers(0, hi))
            zv = int(rng.integers(0, hi))
            if xv or zv:
                break
        x[j] = xv
        z[j] = zv
        phi[j] = rng.uniform(-np.pi, np.pi)
    return x, z, phi


def _segment_masks(p: int, q: int, ends):
    """Masks of one X/Y-Z...Z-X/Y segment on qubits p..q (p < q).

    ``ends`` gives the letters at p and q: 0 for X, 1 for Y.  X sets the x
    bit; Y sets the x and the z bit; the interior p+1..q-1 is Z (z bit only).
    """
    x = (1 << p) | (1 << q)
    z = 0
    for r in range(p + 1, q):
        z |= 1 << r
    if ends[0]:
        z |= 1 << p
    if ends[1]:
        z |= 1 << q
    return x, z


def _draw_term(rng, n: int, w: int):
    """One term of Pauli weight w: a single segment, or (w >= 4, with
    probability 1/2) two disjoint segments of lengths w1 + w2 = w."""
    if w >= 4 and rng.random() < 0.5:
        w1 = int(rng.integers(2, w - 1))  # 2 .. w-2
        w2 = w - w1
        free = n - w
        a, b = sorted(int(v) for v in rng.integers(0, free + 1, size=2))
        p1 = a
        q1 = p1 + w1 - 1
        p2 = q1 + 1 + (b - a)
        q2 = p2 + w2 - 1
        x1, z1 = _segment_masks(p1, q1, rng.integers(0, 2, size=2))
        x2, z2 = _segment_masks(p2, q2, rng.integers(0, 2, size=2))
        return x1 | x2, z1 | z2
    p = int(rng.integers(0, n - w + 1))
    return _segment_masks(p, p + w - 1, rng.integers(0, 2, size=2))


def jw_hamiltonian(n: int, L: int, seed: int = 0):
    """Synthetic Jordan-Wigner-shaped Hamiltonian with L distinct terms.

    Recipe (seeded with ``numpy.random.default_rng(seed)``), per term:
      * bucket: with probability 0.6 the weight is uniform on {2, 3, 4},
        otherwise uniform on {5, ..., n};
      * structure: one X/Y-Z...Z-X/Y segment covering w qubits, or for w >= 4
        with probability 1/2 two disjoint such segments of total weight w,
        placed uniformly;
      * endpoint letters X or Y uniformly; interior letters Z;
      * coefficient: a uniform sign times exp(N(mu=-4, sigma=2)).
    A term equal to one already drawn is redrawn at the same weight (up to
    64 tries) and then at a new weight from the same bucket; only when a
    bucket has no distinct strings left (small n with large L) is the term
    drawn from the other bucket.  Returns (x uint64[L], z uint64[L], h float64[L]).
    """
    if n < 2:
        raise ValueError("need n >= 2")
    rng = np.random.default_rng(seed)
    seen = set()
    xs, zs, hs = [], [], []
    big = list(range(5, n + 1))
    exhausted = {True: False, False: not big}
    while len(xs) < L:
        small_bucket = rng.random() < 0.6 or not big
        got = None
        # a bucket whose distinct strings have run out hands over to the other
        for small in ((True, False) if small_bucket else (False, True)):
            if exhausted[small]:
                continue
            for _ in range(4096):
                w = int(rng.integers(2, 5)) if small else int(rng.choice(big))
                w = min(w, n)
                for _ in range(64):
                    key = _draw_term(rng, n, w)
                    if key not in seen:
                        got = key
                        break
                if got is not None:
                    break
            if got is not None:
                break
            exhausted[small] = True
        if got is None:
            raise ValueError(f"cannot draw {L} distinct terms on {n} qubits")
        seen.add(got)
        xs.append(got[0])
        zs.append(got[1])
        mag = float(np.exp(rng.normal(-4.0, 2.0)))
        hs.append(mag if rng.random() < 0.5 else -mag)
    return (np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64),
            np.array(hs, dtype=np.float64))


def batch_qubit_counts(S: int = 256, lo: int = 16, hi: int = 24, seed: int = 7):
    """Qubit counts of S independent samples, uniform on {lo, ..., hi}."""
    rng = np.random.default_rng(seed)
    return [int(v) for v in rng.integers(lo, hi + 1, size=S)]


# The five workloads: sizes, seeds and schedule parameters.  Each is a plain
# description; builders live in the library (and, independently, the oracle).
WORKLOADS = {
    "random_n14": dict(n=14, M=1000, state_seed=0, rot_seed=1, dtype="c128"),
    "trotter1_n28": dict(n=28, L=2000, ham_seed=0, order=1, t=1.0, steps=10,
                         dtype="c128"),
    "trotter1_n32": dict(n=32, L=5000, ham_seed=0, order=1, t=0.5, steps=4,
                         dtype="c64", check_n=20, check_seed=20),
    "qdrift_batch": dict(S=256, n_lo=16, n_hi=24, n_seed=7, L=500, N=2000, t=1.0,
                         dtype="c64"),
    "partial_n34": dict(n=34, L=8200, ham_seed=0, L_det=200, r=1000, steps=5,
                        t=1.0, dtype="c64", companion_n=33),
}
