"""Robust-phase-estimation signals on top of the rotation engine.

Methods, "Data analysis"; Eq. hamil_split: at step size delta, the
second-order partially randomised formula acts like exp(i delta H~(delta)),
and the frequency that dominates its signal is the lowest eigenvalue of
H~(delta).  Round m of robust phase estimation evaluates

    Z_m = g(delta 2^m) = <psi| exp(i delta H~(delta) 2^m) |psi>,

i.e. 2^m steps of the formula.  The random part takes
r = ceil(kappa lambda_R^2 delta^2 2^M) samples per stage, kappa =
delta / (0.2 pi), and round m draws 2 r 2^m terms from H_R in total (the
factor 2 of the second-order method), so every step here draws 2 r terms.
Deterministic terms are sorted (SUFFIX order), random ones are not.

Every rotation runs in the library's kernels (through the C ABI); this
module only builds schedules, allocates device memory through PyTorch and
post-processes the signal on the host:

* ``samples_per_stage`` -- r from (delta, lambda_R, M);
* ``trotter_error_bound`` -- the commutator bound on the Trotter-error
  prefactor C_gs for the partially randomised split (Methods, "Data
  analysis"), with every deterministic term assumed to anticommute with
  H_R;
* ``signal`` -- Z_0 .. Z_M on the GPU, one random sample per round;
* ``signal_samples`` -- the same rounds with S independent samples each,
  all samples of a round applied by one batched launch sequence
  (prx_batch_run); Z_m is then the sample mean, whose magnitude the finite
  number r of random draws damps (Supplementary, sensitivity to the number
  of random samples);
* ``expected_damping`` -- the exact expected magnitude of that mean for
  commuting terms and a basis eigenstate (a closed form used as a pin);
* ``estimate`` -- the phase of the dominant frequency, unwrapped round by
  round (each round narrows the previous estimate's 2 pi / (delta 2^m)
  ambiguity), as robust phase estimation does with noiseless signals.
"""
from __future__ import annotations

import math

import numpy as np

from . import prx as P


def samples_per_stage(delta: float, lambda_r: float, M: int) -> int:
    """r = ceil(kappa lambda_R^2 delta^2 2^M) with kappa = delta / (0.2 pi)."""
    if delta <= 0 or M < 0:
        raise ValueError("delta must be positive and M non-negative")
    kappa = delta / (0.2 * math.pi)
    return int(math.ceil(kappa * lambda_r * lambda_r * delta * delta * float(2 ** M)))


def _anticommute(x1: int, z1: int, x2: int, z2: int) -> bool:
    return (bin((x1 & z2) ^ (z1 & x2)).count("1") & 1) == 1


def split_weights(h, L_det: int):
    """(D, lambda_R): the L_det terms of largest |h| (ties to the lower
    index) and the 1-norm of the rest, as the partial schedule splits them."""
    h = np.asarray(h, dtype=np.float64)
    order = sorted(range(len(h)), key=lambda l: (-abs(h[l]), l))
    D = sorted(order[:L_det])
    rest = order[L_det:]
    return D, float(np.sum(np.abs(h[rest]))) if rest else 0.0


def trotter_error_bound(x, z, h, L_det: int) -> float:
    """C_gs <= 4 sum_{l in D} |h_l| (sum_{k in D, [P_l, P_k] != 0} |h_k|)^2
    + lambda_R (lambda - lambda_R)^2 + (lambda - lambda_R) lambda_R^2.

    Two Pauli strings either commute or anticommute, so [P_l, P_k] != 0 is
    the symplectic test.  The square on the inner sum follows the general
    commutator bound the specialised form is derived from."""
    x = [int(v) for v in np.asarray(x, dtype=np.uint64)]
    z = [int(v) for v in np.asarray(z, dtype=np.uint64)]
    h = np.asarray(h, dtype=np.float64)
    D, lam_r = split_weights(h, L_det)
    lam = float(np.sum(np.abs(h)))
    det = 0.0
    for l in D:
        inner = sum(abs(h[k]) for k in D if _anticommute(x[l], z[l], x[k], z[k]))
        det += abs(h[l]) * inner * inner
    lam_d = lam - lam_r
    return 4.0 * det + lam_r * lam_d * lam_d + lam_d * lam_r * lam_r


def estimate(Z, delta: float):
    """Dominant frequency of Z_m ~ A exp(i E delta 2^m), m = 0, 1, ...

    Round 0 fixes E in (-pi/delta, pi/delta]; round m picks, among the
    values (arg Z_m + 2 pi k) / (delta 2^m), the one nearest the previous
    estimate.  Returns the estimates after every round (the last is the
    result)."""
    if delta <= 0:
        raise ValueError("delta must be positive")
    est = []
    e = None
    for m, zm in enumerate(Z):
        a = math.atan2(zm.imag, zm.real)
        tm = delta * float(2 ** m)
        if e is None:
            e = a / tm
        else:
            k = round((e * tm - a) / (2.0 * math.pi))
            e = (a + 2.0 * math.pi * k) / tm
        est.append(e)
    return est


def signal(x, z, h, psi0, n: int, dtype: int, delta: float, M: int, L_det: int,
           seed: int = 0, r: int | None = None, kernel: int = P.PRX_AUTO, stream=None):
    """Z_0 .. Z_M for the partially randomised second-order formula.

    psi0: a device tensor (2^n complex64 or complex128 amplitudes), left
    unchanged.  Round m runs 2^m steps of length delta with 2 r random
    draws per step (seed + m for its draws); r defaults to
    samples_per_stage(delta, lambda_R, M).  Returns (Z, r)."""
    import torch

    D, lam_r = split_weights(h, L_det)
    if r is None:
        r = samples_per_stage(delta, lam_r, M) if len(D) < len(h) else 0
    draws = 2 * r if len(D) < len(h) else 0
    H = P.prx_ham_create(n, x, z, h)
    red = torch.empty(P.prx_reduce_workspace_bytes(n), dtype=torch.uint8, device=psi0.device)
    Z = []
    try:
        for m in range(M + 1):
            steps = 2 ** m
            s = P.prx_sched_partial(H, L_det, delta * steps, steps, draws, seed + m,
                                    P.PRX_REORDER_SUFFIX)
            try:
                _, sx, _, _ = P.prx_sched_view(s)
                psi = psi0.clone()
                wsb = P.prx_workspace_bytes(n, dtype, s, kernel)
                ws = torch.empty(max(wsb, 256), dtype=torch.uint8, device=psi0.device)
                P.prx_apply_range(psi, n, dtype, s, 0, len(sx), kernel, ws, stream)
                Z.append(P.prx_overlap(psi0, psi, n, dtype, red, stream))
                del psi, ws
            finally:
                P.prx_sched_destroy(s)
    finally:
        P.prx_ham_destroy(H)
    return Z, r


def sample_seed(seed: int, m: int, s: int) -> int:
    """Seed of sample s in round m of ``signal_samples``."""
    return seed + (m << 20) + s


def signal_samples(x, z, h, psi0, n: int, dtype: int, delta: float, M: int, L_det: int,
                   samples: int, seed: int = 0, r: int | None = None, stream=None):
    """Z_0 .. Z_M as means over `samples` independent random samples per round.

    Round m runs, for every sample s, 2^m steps of length delta with 2 r
    random draws per step, seeded with sample_seed(seed, m, s); the samples
    of a round start from copies of psi0 (a device tensor, left unchanged)
    and run together through prx_batch_run.  Returns (Z, per_sample, r):
    Z[m] the mean of <psi0|psi_s>, per_sample[m] the S overlaps."""
    import torch

    if samples < 1:
        raise ValueError("samples must be >= 1")
    D, lam_r = split_weights(h, L_det)
    if r is None:
        r = samples_per_stage(delta, lam_r, M) if len(D) < len(h) else 0
    draws = 2 * r if len(D) < len(h) else 0
    H = P.prx_ham_create(n, x, z, h)
    red = torch.empty(P.prx_reduce_workspace_bytes(n), dtype=torch.uint8, device=psi0.device)
    Z, per = [], []
    try:
        for m in range(M + 1):
            steps = 2 ** m
            scheds = []
            try:
                for smp in range(samples):
                    scheds.append(P.prx_sched_partial(H, L_det, delta * steps, steps, draws,
                                                      sample_seed(seed, m, smp),
                                                      P.PRX_REORDER_SUFFIX))
                psis = [psi0.clone() for _ in range(samples)]
                b = P.prx_batch_create([n] * samples, scheds, dtype, [0] * samples)
                try:
                    wsb = P.prx_batch_workspace_bytes(b) + 16 * samples + 256
                finally:
                    P.prx_batch_destroy(b)
                ws = torch.empty(wsb, dtype=torch.uint8, device=psi0.device)
                P.prx_batch_run(psis, [n] * samples, scheds, dtype, [0] * samples, ws, stream)
                ov = np.array([P.prx_overlap(psi0, p, n, dtype, red, stream) for p in psis])
                per.append(ov)
                Z.append(complex(ov.mean()))
                del psis, ws
            finally:
                for sc in scheds:
                    P.prx_sched_destroy(sc)
    finally:
        P.prx_ham_destroy(H)
    return Z, per, r


def expected_damping(h, z, b: int, L_det: int, delta: float, m: int, r: int) -> float:
    """|E[Z_m]| for Z-only (commuting) terms and the basis state |b>.

    Every rotation multiplies |b> by a phase, so a sample's Z_m has modulus
    one and only the random phases vary: each of the N = 2 r 2^m draws picks
    term j with probability |h_j| / lambda_R and contributes the phase
    exp(i a sgn(h_j) (-1)^popcount(b & z_j)), a = lambda_R delta / (2 r).
    With mu the probability-weighted mean of those signs, the mean phase of a
    draw has modulus sqrt(cos^2 a + mu^2 sin^2 a), hence
        |E[Z_m]| = (1 - (1 - mu^2) sin^2 a)^(N / 2)."""
    z = [int(v) for v in np.asarray(z, dtype=np.uint64)]
    h = np.asarray(h, dtype=np.float64)
    D, lam_r = split_weights(h, L_det)
    rest = sorted(set(range(len(h))) - set(D))
    if not rest or r == 0:
        return 1.0
    mu = sum(abs(h[j]) * math.copysign(1.0, h[j]) * (-1.0) ** bin(b & z[j]).count("1")
             for j in rest) / lam_r
    a = lam_r * delta / (2 * r)
    N = 2 * r * 2 ** m
    return (1.0 - (1.0 - mu * mu) * math.sin(a) ** 2) ** (N / 2)
