"""Product-formula schedules re-expanded from the paper's definitions.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A schedule is the list of rotations (x_j, z_j, phi_j) in application order:
entry 0 acts on the state first.  For a Hamiltonian H = sum_l h_l P_l with
lambda = sum_l |h_l| (Methods, "Hamiltonian simulation"):

  * first-order Trotter (Eq. define-trotter): exp(i delta H) is approximated
    by the product over l of exp(i delta h_l P_l); with delta = t / S this is
    repeated S times; term l = 1 is applied first;
  * second-order Trotter (the "second-order variant" of the same section):
    per step the terms in order at delta h_l / 2, then in reverse order at
    delta h_l / 2 (symmetric Strang form);
  * qDRIFT (Campbell's random compiler, cited in the same section): N terms
    drawn i.i.d. with probability |h_j| / lambda, each applied at angle
    sgn(h_j) lambda t / N;
  * partially randomised (Eq. hamil_split): H = H_D + H_R with H_D the L_det
    terms of largest |h|; per step the H_D terms forward at delta/2, then r
    qDRIFT draws from H_R at angle sgn(h_j) lambda_R delta / r, then the H_D
    terms in reverse at delta/2;
  * lexicographic ordering of the deterministic terms (Methods, "Data
    analysis"): the terms are stably sorted by (x, z) taken as unsigned
    integers before the deterministic formula is built.

Readings of points the paper leaves open (listed in the design notes):
  time sign e^{+itH}; the product is in application order; the random
  numbers come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), one
  stream per schedule seeded with the given seed, draw i using output i;
  a draw u = (output >> 11) * 2^-53 selects the first index whose running
  FP64 sum of |h| (accumulated left to right) exceeds u times the final sum;
  ties in |h| for the deterministic part go to the lower index.

Angle expressions (kept in this exact operation order so that the library's
schedules can be compared bit for bit):
  first order   phi = (t / S) * h
  second order  phi = ((t / S) * h) * 0.5
  qDRIFT        phi = sgn(h) * ((lambda * t) / N)
  random part   phi = sgn(h) * ((lambda_R * (t / S)) / r)
"""
from __future__ import annotations

import numpy as np

_M64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 as published: a Weyl sequence with increment
    0x9E3779B97F4A7C15 passed through a variant-13 mix (shifts 30, 27, 31;
    multipliers 0xBF58476D1CE4E5B9 and 0x94D049BB133111EB)."""

    def __init__(self, seed: int):
        self.state = seed & _M64

    def next64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _M64
        v = self.state
        v = ((v ^ (v >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        v = ((v ^ (v >> 27)) * 0x94D049BB133111EB) & _M64
        return v ^ (v >> 31)

    def uniform(self) -> float:
        """u in [0, 1) with 53 random bits."""
        return float(self.next64() >> 11) * (2.0 ** -53)


def _sign(h: float) -> float:
    return -1.0 if h < 0 else 1.0


def lambda_of(h) -> float:
    """lambda = sum |h_l|, accumulated left to right in FP64."""
    s = 0.0
    for v in h:
        s += abs(float(v))
    return s


def suffix_order(x, z):
    """Indices of the terms stably sorted by (x, z) as unsigned integers."""
    return sorted(range(len(x)), key=lambda l: (int(x[l]), int(z[l])))


def _as_lists(x, z, h):
    return [int(v) for v in x], [int(v) for v in z], [float(v) for v in h]


def trotter(x, z, h, order: int, t: float, steps: int, suffix: bool = False):
    """First- (order=1) or second-order (order=2) Trotter schedule."""
    x, z, h = _as_lists(x, z, h)
    idx = suffix_order(x, z) if suffix else list(range(len(x)))
    delta = t / steps
    rx, rz, rp = [], [], []
    for _ in range(steps):
        if order == 1:
            for l in idx:
                rx.append(x[l]); rz.append(z[l]); rp.append(delta * h[l])
        elif order == 2:
            for l in idx:
                rx.append(x[l]); rz.append(z[l]); rp.append((delta * h[l]) * 0.5)
            for l in reversed(idx):
                rx.append(x[l]); rz.append(z[l]); rp.append((delta * h[l]) * 0.5)
        else:
            raise ValueError("order must be 1 or 2")
    return _arrays(rx, rz, rp)


def _draw(rng: SplitMix64, prefix) -> int:
    """First index whose running sum of |h| exceeds u * (final sum)."""
    target = rng.uniform() * prefix[-1]
    for j, p in enumerate(prefix):
        if p > target:
            return j
    return len(prefix) - 1  # unreachable for u < 1 and a positive sum


def _prefix(hs):
    out, s = [], 0.0
    for v in hs:
        s += abs(v)
        out.append(s)
    return out


def qdrift(x, z, h, t: float, N: int, seed: int):
    """qDRIFT: N i.i.d. draws with p_j = |h_j| / lambda at angle
    sgn(h_j) * lambda * t / N."""
    x, z, h = _as_lists(x, z, h)
    prefix = _prefix(h)
    lam = prefix[-1]
    rng = SplitMix64(seed)
    ang = (lam * t) / N
    rx, rz, rp = [], [], []
    for _ in range(N):
        j = _draw(rng, prefix)
        rx.append(x[j]); rz.append(z[j]); rp.append(_sign(h[j]) * ang)
    return _arrays(rx, rz, rp)


def partial_split(h, L_det: int):
    """(D, R): D = indices of the L_det largest |h| (ties to the lower
    index) in original order; R = the remaining indices in original order."""
    h = [float(v) for v in h]
    ranked = sorted(range(len(h)), key=lambda l: (-abs(h[l]), l))
    D = sorted(ranked[:L_det])
    inD = set(D)
    R = [l for l in range(len(h)) if l not in inD]
    return D, R


def partial(x, z, h, L_det: int, t: float, steps: int, r: int, seed: int,
            suffix: bool = False):
    """Partially randomised product formula (second-order deterministic part,
    qDRIFT-sampled random part in the middle of every step)."""
    x, z, h = _as_lists(x, z, h)
    D, R = partial_split(h, L_det)
    if suffix:
        D = [D[i] for i in suffix_order([x[l] for l in D], [z[l] for l in D])]
    delta = t / steps
    prefR = _prefix([h[l] for l in R])
    lamR = prefR[-1] if R else 0.0
    ang = (lamR * delta) / r if r > 0 else 0.0
    rng = SplitMix64(seed)
    rx, rz, rp = [], [], []
    for _ in range(steps):
        for l in D:
            rx.append(x[l]); rz.append(z[l]); rp.append((delta * h[l]) * 0.5)
        if R:
            for _ in range(r):
                j = R[_draw(rng, prefR)]
                rx.append(x[j]); rz.append(z[j]); rp.append(_sign(h[j]) * ang)
        for l in reversed(D):
            rx.append(x[l]); rz.append(z[l]); rp.append((delta * h[l]) * 0.5)
    return _arrays(rx, rz, rp)


def _arrays(rx, rz, rp):
    return (np.array(rx, dtype=np.uint64), np.array(rz, dtype=np.uint64),
            np.array(rp, dtype=np.float64))
