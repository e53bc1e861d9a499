"""Pins that tie the CPU oracle to the paper and to mathematics, not to itself.

Each test names what fixes the expected value: the paper's worked example,
dense matrices built from textbook Pauli matrices and scipy's matrix
exponential, closed forms, invariants, published generator outputs, or
statistics with known distributions.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

import synth
from oracle import pauli, schedules, statevector as sv

# Textbook Pauli matrices.
_I2 = np.eye(2, dtype=complex)
_X = np.array([[0, 1], [1, 0]], dtype=complex)
_Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
_Z = np.array([[1, 0], [0, -1]], dtype=complex)
_MAT = {"I": _I2, "X": _X, "Y": _Y, "Z": _Z}


def dense_pauli(label: str) -> np.ndarray:
    """Kronecker product; character q acts on qubit q = bit q (LSB first),
    so the last character is the leftmost Kronecker factor."""
    m = np.array([[1.0 + 0j]])
    for ch in label:
        m = np.kron(_MAT[ch], m)
    return m


def letters(x: int, z: int, n: int) -> str:
    # decoding written independently of oracle.pauli (x bit: X/Y, z bit: Y/Z)
    out = []
    for q in range(n):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        out.append({(0, 0): "I", (1, 0): "X", (1, 1): "Y", (0, 1): "Z"}[(xb, zb)])
    return "".join(out)


def dense_rotation(x, z, phi, n):
    return scipy.linalg.expm(1j * phi * dense_pauli(letters(x, z, n)))


def rand_state(n, seed):
    return synth.gaussian_state(n, seed)


# ---------------------------------------------------------------- encoding

def test_encoding_worked_example(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "encoding_example.json")))
    x, z = pauli.label_to_masks("".join(g["factors"]))
    assert (x, z) == (g["p1"], g["p2"])
    assert pauli.masks_to_label(x, z, 3) == "".join(g["factors"])


# ---------------------------------------------------------- Pauli action

@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_pauli_action_all_strings_dense(n):
    psi = rand_state(n, 3)
    for x in range(1 << n):
        for z in range(1 << n):
            ref = dense_pauli(letters(x, z, n)) @ psi
            np.testing.assert_allclose(sv.pauli_apply(x, z, psi), ref, atol=1e-15)
            np.testing.assert_allclose(sv.c_pauli_apply(x, z, psi), ref, atol=1e-15)


def test_destination_sign_form_is_wrong_for_odd_y():
    """The form with the sign taken from the destination index equals P^T,
    which differs from P exactly for strings with an odd number of Y's."""
    n = 3
    psi = rand_state(n, 4)
    N = 1 << n
    bad = 0
    for x in range(N):
        for z in range(N):
            nY = bin(x & z).count("1")
            alt = np.array([(1j ** nY) * (-1) ** bin(k & z).count("1") * psi[k ^ x]
                            for k in range(N)])
            same = np.allclose(alt, sv.pauli_apply(x, z, psi), atol=1e-14)
            assert same == (nY % 2 == 0)
            bad += not same
    assert bad == 28


# ------------------------------------------------------------ rotations

@pytest.mark.parametrize("n", [1, 3, 6])
def test_single_rotation_expm_and_closed_form(n):
    rng = np.random.default_rng(5)
    psi = rand_state(n, 5)
    for _ in range(40):
        x, z = int(rng.integers(0, 1 << n)), int(rng.integers(0, 1 << n))
        phi = float(rng.uniform(-np.pi, np.pi))
        P = dense_pauli(letters(x, z, n))
        ref = scipy.linalg.expm(1j * phi * P) @ psi
        closed = (math.cos(phi) * np.eye(1 << n) + 1j * math.sin(phi) * P) @ psi
        np.testing.assert_allclose(closed, ref, atol=1e-13)
        out = sv.apply_rotations(psi, [x], [z], [phi])
        np.testing.assert_allclose(out, ref, atol=1e-13)
        np.testing.assert_allclose(sv.c_apply_rotations(psi, [x], [z], [phi]), ref,
                                   atol=1e-13)


@pytest.mark.parametrize("n,M", [(5, 30), (8, 12)])
def test_sequence_against_dense_product(n, M):
    x, z, phi = synth.random_pauli_rotations(n, M, seed=11)
    psi = rand_state(n, 6)
    U = np.eye(1 << n, dtype=complex)
    for j in range(M):  # entry 0 acts first
        U = dense_rotation(int(x[j]), int(z[j]), float(phi[j]), n) @ U
    ref = U @ psi
    np.testing.assert_allclose(sv.apply_rotations(psi, x, z, phi), ref, atol=1e-12)
    np.testing.assert_allclose(sv.c_apply_rotations(psi, x, z, phi), ref, atol=1e-12)


def test_norm_preserved_and_numpy_equals_c():
    n, M = 10, 300
    x, z, phi = synth.random_pauli_rotations(n, M, seed=12)
    psi = rand_state(n, 7)
    a = sv.apply_rotations(psi, x, z, phi)
    b = sv.c_apply_rotations(psi, x, z, phi)
    assert abs(sv.norm2(a) - 1.0) < 1e-13
    assert abs(sv.c_norm2(b) - 1.0) < 1e-13
    np.testing.assert_allclose(a, b, atol=1e-13)


def test_rotation_then_inverse_is_identity():
    n = 7
    x, z, phi = synth.random_pauli_rotations(n, 50, seed=13)
    psi = rand_state(n, 8)
    for j in range(50):
        out = sv.apply_rotations(psi, [x[j], x[j]], [z[j], z[j]], [phi[j], -phi[j]])
        np.testing.assert_allclose(out, psi, atol=1e-15)
    # the whole list, then the reversed list with negated angles
    fwd = sv.c_apply_rotations(psi, x, z, phi)
    back = sv.c_apply_rotations(fwd, x[::-1], z[::-1], -phi[::-1])
    np.testing.assert_allclose(back, psi, atol=1e-13)


def test_z_only_closed_form():
    n, M = 9, 40
    rng = np.random.default_rng(14)
    z = rng.integers(0, 1 << n, size=M).astype(np.uint64)
    x = np.zeros(M, dtype=np.uint64)
    phi = rng.uniform(-3, 3, size=M)
    psi = rand_state(n, 9)
    k = np.arange(1 << n, dtype=np.uint64)
    ang = np.zeros(1 << n)
    for j in range(M):
        ang += phi[j] * (1.0 - 2.0 * (np.bitwise_count(k & z[j]) & 1).astype(np.float64))
    ref = psi * np.exp(1j * ang)
    np.testing.assert_allclose(sv.apply_rotations(psi, x, z, phi), ref, atol=1e-13)
    np.testing.assert_allclose(sv.c_apply_rotations(psi, x, z, phi), ref, atol=1e-13)


def test_identity_string_is_global_phase():
    psi = rand_state(4, 10)
    out = sv.apply_rotations(psi, [0], [0], [0.3])
    np.testing.assert_allclose(out, np.exp(0.3j) * psi, atol=1e-15)


def _commutes_dense(a, b, n):
    A = dense_pauli(letters(*a, n))
    B = dense_pauli(letters(*b, n))
    return np.allclose(A @ B, B @ A)


def test_commuting_order_invariance():
    n = 6
    rng = np.random.default_rng(15)
    chosen = []
    while len(chosen) < 8:
        cand = (int(rng.integers(0, 1 << n)), int(rng.integers(0, 1 << n)))
        if cand == (0, 0):
            continue
        if all(_commutes_dense(cand, c, n) for c in chosen):
            chosen.append(cand)
    phi = rng.uniform(-2, 2, size=len(chosen))
    psi = rand_state(n, 11)
    x = [c[0] for c in chosen]
    z = [c[1] for c in chosen]
    ref = sv.apply_rotations(psi, x, z, phi)
    for _ in range(5):
        p = rng.permutation(len(chosen))
        out = sv.c_apply_rotations(psi, [x[i] for i in p], [z[i] for i in p], phi[p])
        np.testing.assert_allclose(out, ref, atol=1e-13)


# ---------------------------------------------- Eq. (1): common suffix

def test_common_suffix_identity_dense_and_buffer_recipe():
    """Eq. (core): a run of rotations P_l (x) Q equals prod e^{+i phi P_l}
    (x) (I+Q)/2 + prod e^{-i phi P_l} (x) (I-Q)/2, and the three-step buffer
    recipe of the Supplementary Methods reproduces it."""
    lo, hi = 4, 2
    n = lo + hi
    rng = np.random.default_rng(16)
    Lr = 6
    Ps = [(int(rng.integers(1, 1 << lo)), int(rng.integers(0, 1 << lo))) for _ in range(Lr)]
    Q = (0b01, 0b11)  # letters on the upper qubits: Y on the first, Z on the second
    phi = rng.uniform(-1.5, 1.5, size=Lr)
    Qm = dense_pauli(letters(*Q, hi))
    Iq = np.eye(1 << hi)
    Up = np.eye(1 << lo, dtype=complex)
    Um = np.eye(1 << lo, dtype=complex)
    lhs = np.eye(1 << n, dtype=complex)
    for (px, pz), f in zip(Ps, phi):
        Pm = dense_pauli(letters(px, pz, lo))
        Up = scipy.linalg.expm(1j * f * Pm) @ Up
        Um = scipy.linalg.expm(-1j * f * Pm) @ Um
        lhs = scipy.linalg.expm(1j * f * np.kron(Qm, Pm)) @ lhs
    rhs = np.kron((Iq + Qm) / 2, Up) + np.kron((Iq - Qm) / 2, Um)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)

    # oracle applied sequentially to the full strings
    psi = rand_state(n, 12)
    fx = [px | (Q[0] << lo) for px, _ in Ps]
    fz = [pz | (Q[1] << lo) for _, pz in Ps]
    seq = sv.apply_rotations(psi, fx, fz, phi)
    np.testing.assert_allclose(seq, rhs @ psi, atol=1e-12)
    # three steps: psi' = (I (x) Q) psi; A = (psi+psi')/sqrt2, B = (psi-psi')/sqrt2;
    # rotations with +phi on A and -phi on B (lower qubits only); (A+B)/sqrt2.
    psi_p = sv.pauli_apply(Q[0] << lo, Q[1] << lo, psi)
    A = (psi + psi_p) / math.sqrt(2)
    B = (psi - psi_p) / math.sqrt(2)
    A = sv.apply_rotations(A, [p[0] for p in Ps], [p[1] for p in Ps], phi)
    B = sv.apply_rotations(B, [p[0] for p in Ps], [p[1] for p in Ps], -phi)
    np.testing.assert_allclose((A + B) / math.sqrt(2), seq, atol=1e-12)


def test_upper_pauli_phase_relation():
    """For a string on the upper qubits, P|k> = w_k |k'> is a bijection
    k -> k' with w_{k'} = conj(w_k) (Supplementary Methods)."""
    m = 4
    for x in range(1 << m):
        for z in range(1 << m):
            P = dense_pauli(letters(x, z, m))
            seen = set()
            w = {}
            for k in range(1 << m):
                col = P[:, k]
                kp = int(np.flatnonzero(np.abs(col) > 0.5)[0])
                w[k] = (kp, col[kp])
                seen.add(kp)
                assert kp == k ^ x
            assert len(seen) == 1 << m
            for k, (kp, wk) in w.items():
                assert abs(w[kp][1] - np.conj(wk)) < 1e-15


# --------------------------------------------------------- reductions

def test_overlap_exact_rational_and_basis():
    n = 5
    rng = np.random.default_rng(17)
    # dyadic values so that the exact sum is representable
    a = (rng.integers(-2**20, 2**20, size=(2, 1 << n)) / 2**20)
    b = (rng.integers(-2**20, 2**20, size=(2, 1 << n)) / 2**20)
    p0 = a[0] + 1j * a[1]
    p1 = b[0] + 1j * b[1]
    re = sum(Fraction(float(a[0, k])) * Fraction(float(b[0, k])) +
             Fraction(float(a[1, k])) * Fraction(float(b[1, k])) for k in range(1 << n))
    im = sum(Fraction(float(a[0, k])) * Fraction(float(b[1, k])) -
             Fraction(float(a[1, k])) * Fraction(float(b[0, k])) for k in range(1 << n))
    for ov in (sv.overlap(p0, p1), sv.c_overlap(p0, p1)):
        assert ov.real == float(re) and ov.imag == float(im)
    nn = sum(Fraction(float(a[0, k])) ** 2 + Fraction(float(a[1, k])) ** 2
             for k in range(1 << n))
    assert sv.norm2(p0) == float(nn) and sv.c_norm2(p0) == float(nn)
    # basis bra picks one amplitude
    e = np.zeros(1 << n, dtype=complex)
    e[9] = 1
    assert sv.c_overlap(e, p1) == p1[9]


def test_compensated_sum_beats_naive_on_cancellation():
    N = 1 << 12
    v = np.zeros(N, dtype=complex)
    v[0] = 1e16
    v[1:2049] = 1.0
    v[2049] = -1e16
    e = np.ones(N, dtype=complex)
    assert sv.c_overlap(e, v).real == 2048.0
    assert sv.overlap(e, v).real == 2048.0


# --------------------------------------------------------------- PRNG

def test_splitmix64_published_outputs(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "splitmix64.json")))
    r = schedules.SplitMix64(g["seed"])
    assert [r.next64() for _ in range(5)] == [int(v) for v in g["outputs"]]


def test_qdrift_sampler_chi_square():
    h = np.array([0.5, -0.1, 0.02, 1.3, -0.7, 0.08, 0.0, 0.25])
    x = np.arange(1, 9, dtype=np.uint64)
    z = np.zeros(8, dtype=np.uint64)
    N = 200_000
    rx, _, rp = schedules.qdrift(x, z, h, t=1.0, N=N, seed=99)
    counts = np.bincount(rx.astype(np.int64) - 1, minlength=8)
    assert counts[6] == 0  # a zero coefficient is never drawn
    p = np.abs(h) / np.abs(h).sum()
    keep = p > 0
    chi2 = float(np.sum((counts[keep] - N * p[keep]) ** 2 / (N * p[keep])))
    assert scipy.stats.chi2.sf(chi2, df=int(keep.sum()) - 1) > 1e-4
    lam = float(np.abs(h).sum())
    # angle magnitude lambda t / N, sign of the drawn coefficient
    assert np.all(np.abs(np.abs(rp) - lam / N) <= 1e-18)
    assert np.all(np.sign(rp) == np.sign(h[rx.astype(np.int64) - 1]))


# ------------------------------------------------------- product formulas

def _small_h(n, L, seed):
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 1 << n, size=L).astype(np.uint64)
    z = rng.integers(0, 1 << n, size=L).astype(np.uint64)
    h = rng.normal(0, 0.5, size=L)
    return x, z, h


def _dense_h(x, z, h, n):
    return sum(float(h[l]) * dense_pauli(letters(int(x[l]), int(z[l]), n))
               for l in range(len(h)))


def test_trotter_exact_for_commuting_hamiltonian():
    n = 6
    rng = np.random.default_rng(18)
    z = rng.integers(1, 1 << n, size=10).astype(np.uint64)
    x = np.zeros(10, dtype=np.uint64)
    h = rng.normal(size=10)
    psi = rand_state(n, 13)
    exact = scipy.linalg.expm(1j * 0.8 * _dense_h(x, z, h, n)) @ psi
    for order in (1, 2):
        rx, rz, rp = schedules.trotter(x, z, h, order, 0.8, 3)
        np.testing.assert_allclose(sv.apply_rotations(psi, rx, rz, rp), exact, atol=1e-13)


@pytest.mark.parametrize("order,slope", [(1, 1.0), (2, 2.0)])
def test_trotter_error_slope(order, slope):
    n = 5
    x, z, h = _small_h(n, 12, 19)
    psi = rand_state(n, 14)
    t = 1.0
    exact = scipy.linalg.expm(1j * t * _dense_h(x, z, h, n)) @ psi
    errs = []
    Ss = [8, 16, 32, 64]
    for S in Ss:
        rx, rz, rp = schedules.trotter(x, z, h, order, t, S)
        errs.append(np.linalg.norm(sv.apply_rotations(psi, rx, rz, rp) - exact))
    fit = np.polyfit(np.log(1.0 / np.array(Ss)), np.log(errs), 1)[0]
    assert abs(fit - slope) < 0.15, (fit, errs)


def test_trotter_time_sign_and_order():
    """e^{+itH}: one first-order step of a single term is e^{+i t h P}."""
    n = 3
    psi = rand_state(n, 15)
    rx, rz, rp = schedules.trotter([0b011], [0b010], [0.7], 1, 0.4, 1)
    ref = scipy.linalg.expm(1j * 0.4 * 0.7 * dense_pauli(letters(0b011, 0b010, n))) @ psi
    np.testing.assert_allclose(sv.apply_rotations(psi, rx, rz, rp), ref, atol=1e-14)


def test_second_order_step_is_time_symmetric():
    n = 4
    x, z, h = _small_h(n, 7, 20)
    psi = rand_state(n, 16)
    fx, fz, fp = schedules.trotter(x, z, h, 2, 0.3, 1)
    bx, bz, bp = schedules.trotter(x, z, h, 2, -0.3, 1)
    out = sv.apply_rotations(sv.apply_rotations(psi, fx, fz, fp), bx, bz, bp)
    np.testing.assert_allclose(out, psi, atol=1e-14)


def test_qdrift_mean_overlap_converges():
    n = 4
    x, z, h = _small_h(n, 6, 21)
    psi = rand_state(n, 17)
    t = 0.5
    exact = np.vdot(psi, scipy.linalg.expm(1j * t * _dense_h(x, z, h, n)) @ psi)
    lam = float(np.abs(h).sum())
    N = 400
    vals = []
    for seed in range(300):
        rx, rz, rp = schedules.qdrift(x, z, h, t, N, seed)
        vals.append(np.vdot(psi, sv.apply_rotations(psi, rx, rz, rp)))
    mean = np.mean(vals)
    se = np.std(vals) / math.sqrt(len(vals))
    bias = (lam * t) ** 2 / N
    assert abs(mean - exact) < 4 * se + 2 * bias, (mean, exact, se, bias)


def test_partial_split_and_limits():
    n = 4
    x, z, h = _small_h(n, 9, 22)
    D, R = schedules.partial_split(h, 3)
    top = sorted(range(9), key=lambda l: -abs(h[l]))[:3]
    assert sorted(D) == sorted(top) and sorted(D + R) == list(range(9))
    # with every term deterministic the formula is second-order Trotter
    px, pz, pp = schedules.partial(x, z, h, 9, 0.6, 3, 5, seed=1)
    tx, tz, tp = schedules.trotter(x, z, h, 2, 0.6, 3)
    assert np.array_equal(px, tx) and np.array_equal(pz, tz) and np.array_equal(pp, tp)
    # layout: per step |D| forward, r random, |D| reversed
    px, pz, pp = schedules.partial(x, z, h, 3, 0.6, 2, 5, seed=1)
    assert len(px) == 2 * (2 * 3 + 5)
    assert np.array_equal(px[:3], px[8:11][::-1])


def test_partial_mean_overlap_converges():
    n = 4
    x, z, h = _small_h(n, 8, 23)
    psi = rand_state(n, 18)
    t = 0.5
    exact = np.vdot(psi, scipy.linalg.expm(1j * t * _dense_h(x, z, h, n)) @ psi)
    vals = []
    for seed in range(200):
        rx, rz, rp = schedules.partial(x, z, h, 3, t, 4, 60, seed)
        vals.append(np.vdot(psi, sv.apply_rotations(psi, rx, rz, rp)))
    mean = np.mean(vals)
    se = np.std(vals) / math.sqrt(len(vals))
    D, R = schedules.partial_split(h, 3)
    lamR = float(np.abs(h[R]).sum())
    bias = (lamR * t) ** 2 / (4 * 60) + 0.05 * (t / 4) ** 2 * float(np.abs(h).sum()) ** 2
    assert abs(mean - exact) < 4 * se + bias, (mean, exact, se, bias)


def test_suffix_order_groups_high_bits():
    x = np.array([0b1100, 0b0011, 0b1000, 0b0100, 0b1100], dtype=np.uint64)
    z = np.array([3, 0, 0, 1, 1], dtype=np.uint64)
    order = schedules.suffix_order(x, z)
    assert order == [1, 3, 2, 4, 0]
    hi = [int(x[l]) >> 2 for l in order]
    # equal high parts are contiguous
    runs = [hi[0]] + [b for a, b in zip(hi, hi[1:]) if a != b]
    assert len(runs) == len(set(hi))
