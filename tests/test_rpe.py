"""Robust-phase-estimation helpers on the host: estimator, sample count and
the Trotter-error bound, pinned by closed forms (no GPU)."""
import math

import numpy as np
import pytest

from paper_2504_17881_amd import rpe


@pytest.mark.parametrize("E", [0.3, -1.7, 2.9, -3.1, 12.345])
def test_estimate_recovers_exact_frequency(E):
    delta, M = 0.25, 12
    if abs(E) >= math.pi / delta:
        pytest.skip("outside the unambiguous range of round 0")
    Z = [complex(math.cos(E * delta * 2 ** m), math.sin(E * delta * 2 ** m)) for m in range(M + 1)]
    est = rpe.estimate(Z, delta)
    assert abs(est[-1] - E) <= 1e-9 * max(1.0, abs(E))


def test_estimate_with_a_weaker_second_frequency():
    """Z_m = a1 e^{i E1 t} + a2 e^{i E2 t}: each round's phase is off by at
    most asin(a2/a1) < pi/2, so unwrapping never slips and the final error
    is at most asin(a2/a1) / (delta 2^M)."""
    rng = np.random.default_rng(3)
    delta, M = 0.3, 14
    for _ in range(20):
        E1, E2 = rng.uniform(-3, 3, size=2)
        a1, a2 = 0.75, 0.25
        Z = [a1 * complex(math.cos(E1 * delta * 2 ** m), math.sin(E1 * delta * 2 ** m)) +
             a2 * complex(math.cos(E2 * delta * 2 ** m), math.sin(E2 * delta * 2 ** m))
             for m in range(M + 1)]
        est = rpe.estimate(Z, delta)
        assert abs(est[-1] - E1) <= math.asin(a2 / a1) / (delta * 2 ** M) + 1e-12


def test_samples_per_stage():
    # kappa = delta / (0.2 pi); r = ceil(kappa lambda_R^2 delta^2 2^M)
    delta, lam, M = 0.1, 3.0, 10
    want = math.ceil(delta / (0.2 * math.pi) * lam * lam * delta * delta * 1024)
    assert rpe.samples_per_stage(delta, lam, M) == want == 15
    assert rpe.samples_per_stage(0.5, 0.0, 5) == 0
    with pytest.raises(ValueError):
        rpe.samples_per_stage(0.0, 1.0, 3)


def test_trotter_error_bound_single_qubit_pair():
    """X (h = a) and Z (h = b) anticommute.  All deterministic:
    4 (a b^2 + b a^2).  D = {X} (a > b), R = {Z}: the deterministic sum is
    empty and the split terms give b a^2 + a b^2."""
    a, b = 0.7, 0.2
    x = np.array([1, 0], dtype=np.uint64)
    z = np.array([0, 1], dtype=np.uint64)
    h = np.array([a, -b])
    assert rpe.trotter_error_bound(x, z, h, 2) == pytest.approx(4 * (a * b * b + b * a * a))
    assert rpe.trotter_error_bound(x, z, h, 1) == pytest.approx(b * a * a + a * b * b)


def test_trotter_error_bound_commuting_terms_vanish():
    # Z-only strings commute: no deterministic contribution, no random part
    rng = np.random.default_rng(0)
    z = rng.integers(1, 1 << 6, size=12).astype(np.uint64)
    x = np.zeros(12, dtype=np.uint64)
    h = rng.normal(size=12)
    assert rpe.trotter_error_bound(x, z, h, 12) == 0.0


def test_split_weights_matches_schedule_split():
    from oracle.schedules import partial_split
    rng = np.random.default_rng(1)
    h = rng.normal(size=40)
    h[5] = h[7]  # a tie
    for L_det in (0, 1, 7, 40):
        D, lam_r = rpe.split_weights(h, L_det)
        D2, R2 = partial_split(h, L_det)
        assert D == D2
        assert lam_r == pytest.approx(float(np.sum(np.abs(h[R2]))) if R2 else 0.0)


def _zonly(n, L, seed):
    rng = np.random.default_rng(seed)
    z = rng.integers(1, 1 << n, size=L).astype(np.uint64)
    return np.zeros(L, dtype=np.uint64), z, rng.normal(scale=0.5, size=L)


@pytest.mark.parametrize("r", [1, 16])
def test_damping_closed_form_against_oracle_samples(r):
    """Supplementary, sensitivity to the number of random samples: fewer
    random draws damp the sample-mean signal.  For Z-only terms and a basis
    state every sample is a pure phase, and the mean over many oracle runs
    (schedules re-expanded by the oracle, states by its numpy loop) matches the
    closed form of rpe.expected_damping within the sampling error; the
    closed form itself falls as r shrinks."""
    import synth
    from oracle import schedules as osch
    from oracle import statevector as sv
    n, L, L_det, delta, m, S = 6, 12, 4, 0.5, 3, 1000
    x, z, h = _zonly(n, L, 3)
    b = synth.basis_index(n)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[b] = 1.0
    acc = 0.0 + 0.0j
    for s in range(S):
        rx, rz, rp = osch.partial(x, z, h, L_det, delta * 2 ** m, 2 ** m, 2 * r,
                                  rpe.sample_seed(9, m, s), suffix=True)
        out = sv.apply_rotations(psi0, rx, rz, rp)
        assert abs(abs(out[b]) - 1.0) <= 1e-12
        acc += out[b]
    mean = abs(acc / S)
    want = rpe.expected_damping(h, z, b, L_det, delta, m, r)
    assert abs(mean - want) <= 0.1, (mean, want)
    assert rpe.expected_damping(h, z, b, L_det, delta, m, 1) < \
        rpe.expected_damping(h, z, b, L_det, delta, m, 4) < \
        rpe.expected_damping(h, z, b, L_det, delta, m, 16) < 1.0


def test_damping_without_random_part_is_one():
    x, z, h = _zonly(6, 12, 3)
    assert rpe.expected_damping(h, z, 7, 12, 0.5, 4, 0) == 1.0
