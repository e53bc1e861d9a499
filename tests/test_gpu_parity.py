"""GPU parity: the HIP kernels through the C ABI against the CPU oracle.

Tolerances:
  * complex128: relative 2-norm error of the state and |delta overlap| at
    most 1e-12 (FP64 rounding after ~10^3 rotations is ~1e-14);
  * complex64: relative 2-norm error at most 8 * eps32 * sqrt(M) with
    eps32 = 2^-24 (a random walk of per-rotation rounding errors of a few
    ulps), and |delta overlap| at most 1e-4 at 10^4 rotations.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import statevector as sv
from paper_2504_17881_amd import prx as P
from gpu_util import (apply, basis_state, overlap, rel_err, to_dev, to_host, workspace)

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24


def c64_tol(M):
    return 8 * EPS32 * math.sqrt(max(M, 1)) + 1e-6


def _run_both(n, x, z, phi, psi0, dtype, kernel, opts=None):
    s = P.prx_sched_from_rotations(n, x, z, phi)
    t = to_dev(psi0, dtype)
    info = apply(t, n, dtype, s, kernel, opts=opts)
    P.prx_sched_destroy(s)
    return t, info


@pytest.mark.parametrize("kernel", [P.PRX_PLAIN, P.PRX_FUSED])
def test_random_rotations_n14_c128(kernel):
    """Random strings over {I,X,Y,Z}^14, angles in [-pi, pi], Gaussian state."""
    w = synth.WORKLOADS["random_n14"]
    n, M = w["n"], w["M"]
    x, z, phi = synth.random_pauli_rotations(n, M, seed=w["rot_seed"])
    psi0 = synth.gaussian_state(n, w["state_seed"])
    ref = sv.c_apply_rotations(psi0, x, z, phi)
    print(f"[random_n14 kernel={kernel}]", flush=True)
    t, info = _run_both(n, x, z, phi, psi0, P.PRX_C128, kernel)
    out = to_host(t)
    assert rel_err(out, ref) <= 1e-12
    ov = overlap(to_dev(psi0, P.PRX_C128), t, n, P.PRX_C128)
    assert abs(ov - sv.c_overlap(psi0, ref)) <= 1e-12


def test_random_rotations_n14_c64():
    w = synth.WORKLOADS["random_n14"]
    n, M = w["n"], w["M"]
    x, z, phi = synth.random_pauli_rotations(n, M, seed=w["rot_seed"])
    psi0 = synth.gaussian_state(n, w["state_seed"])
    ref = sv.c_apply_rotations(psi0, x, z, phi)
    for kernel in (P.PRX_PLAIN, P.PRX_FUSED):
        t, _ = _run_both(n, x, z, phi, psi0, P.PRX_C64, kernel)
        assert rel_err(to_host(t), ref) <= c64_tol(M)


SHAPES = [
    dict(tile_qubits=10, chunk_rank=3),
    dict(tile_qubits=10, chunk_rank=4),
    dict(tile_qubits=11, chunk_rank=4, max_virtual=1),
    dict(tile_qubits=12, chunk_rank=4, max_virtual=2),
    dict(tile_qubits=12, chunk_rank=5),
    dict(tile_qubits=13, chunk_rank=4, max_virtual=2, span_max=2),
    dict(tile_qubits=14, chunk_rank=4, span_max=2),
    dict(tile_qubits=10, chunk_rank=4, max_virtual=5, span_max=2),
    dict(tile_qubits=11, chunk_rank=4, max_virtual=4, span_max=2),
    dict(span_max=1),
    dict(span_max=2),
    dict(span_max=3),
    dict(span_max=5),
    dict(max_fuse=3),
    dict(commuting=1),
]


@pytest.mark.parametrize("opts", SHAPES)
@pytest.mark.parametrize("dtype", [P.PRX_C128, P.PRX_C64])
def test_fused_shapes_jw_trotter(opts, dtype):
    """Every instantiated tile shape, span rank and planner option against
    the oracle on a SUFFIX-ordered JW Trotter run (tiles and spans mixed)."""
    if dtype == P.PRX_C128 and opts.get("tile_qubits", 0) >= 14:
        pytest.skip("complex128 tiles above 13 qubits are not built (LDS budget)")
    n = 15
    x, z, h = synth.jw_hamiltonian(n, 400, 11)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_trotter(H, 1, 3.0, 2, P.PRX_REORDER_SUFFIX)
    _, rx, rz, rp = P.prx_sched_view(s)
    psi0 = synth.gaussian_state(n, 12)
    ref = sv.c_apply_rotations(psi0, rx, rz, rp)
    print(f"[shapes {opts} dtype={dtype}]", flush=True)
    t = to_dev(psi0, dtype)
    info = apply(t, n, dtype, s, P.PRX_FUSED, opts=opts)
    err = rel_err(to_host(t), ref)
    tol = 1e-12 if dtype == P.PRX_C128 else c64_tol(len(rx))
    assert err <= tol, (err, info)
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


@pytest.mark.parametrize("n,B,g,dtype", [
    (20, 12, 6, P.PRX_C64), (20, 12, 8, P.PRX_C64), (20, 11, 6, P.PRX_C128),
    (20, 11, 8, P.PRX_C128), (22, 13, 8, P.PRX_C64), (24, 14, 10, P.PRX_C64),
    (22, 13, 9, P.PRX_C128)])
def test_many_virtual_qubits(n, B, g, dtype):
    """Tile-sets of 2^g tiles with as few as 16 contiguous amplitudes (the
    128 KiB frames, 14 qubits at complex64 and 13 at complex128, run
    persistent workgroups), spans limited so that tiles take the high X
    parts."""
    x, z, h = synth.jw_hamiltonian(n, 300 if n < 24 else 200, 21)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_trotter(H, 1, 2.0, 1, P.PRX_REORDER_SUFFIX)
    _, rx, rz, rp = P.prx_sched_view(s)
    psi0 = synth.gaussian_state(n, 22)
    ref = sv.c_apply_rotations(psi0, rx, rz, rp)
    opts = dict(tile_qubits=B, chunk_rank=4, max_virtual=g, span_max=2, max_fuse=128)
    print(f"[many virtual n={n} B={B} g={g} dtype={dtype}]", flush=True)
    pl = P.prx_plan_create(s, n, dtype, 0, len(rx), P.PRX_FUSED, opts)
    gs = [P.prx_plan_pass(pl, i)["g"] for i in range(P.prx_plan_get_info(pl)["passes"])]
    assert max(gs) >= min(g, 5)
    P.prx_plan_destroy(pl)
    t = to_dev(psi0, dtype)
    info = apply(t, n, dtype, s, P.PRX_FUSED, opts=opts)
    err = rel_err(to_host(t), ref)
    tol = 1e-12 if dtype == P.PRX_C128 else c64_tol(len(rx))
    assert err <= tol, (err, info)
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 9, 11, 13])
@pytest.mark.parametrize("kernel", [P.PRX_PLAIN, P.PRX_FUSED])
def test_small_and_ragged_sizes(n, kernel):
    """Sizes below one tile, a single workgroup, and just above."""
    M = 60
    x, z, phi = synth.random_pauli_rotations(n, M, seed=100 + n)
    psi0 = synth.gaussian_state(n, n)
    ref = sv.c_apply_rotations(psi0, x, z, phi)
    t, _ = _run_both(n, x, z, phi, psi0, P.PRX_C128, kernel)
    assert rel_err(to_host(t), ref) <= 1e-12


def test_diagonal_identity_and_large_angles():
    n = 12
    rng = np.random.default_rng(5)
    z = rng.integers(0, 1 << n, size=30).astype(np.uint64)
    x = np.zeros(30, dtype=np.uint64)
    x[::3] = rng.integers(1, 1 << n, size=10).astype(np.uint64)
    z[4] = 0
    x[4] = 0  # identity string: global phase
    phi = rng.uniform(-3.1, 3.1, size=30)
    phi[7] = math.pi / 2  # cos = 0: split into two half angles by fused plans
    phi[8] = -math.pi / 2
    phi[9] = math.pi
    psi0 = synth.gaussian_state(n, 9)
    ref = sv.c_apply_rotations(psi0, x, z, phi)
    for kernel in (P.PRX_PLAIN, P.PRX_FUSED):
        t, _ = _run_both(n, x, z, phi, psi0, P.PRX_C128, kernel)
        assert rel_err(to_host(t), ref) <= 1e-12


@pytest.mark.parametrize("B", [12, 14])
def test_diagonal_records_inside_complex64_tile_chunks(B):
    """Z-only rotations interleaved with others (alone, in runs of three,
    first or last in a chunk) inside complex64 tile chunks, where the
    threaded rotation loop stops at each diagonal record, leaves it to the
    compiled path and resumes after it; 12-qubit tile-sets (five workgroups
    per CU) and the persistent 14-qubit ones."""
    n, M = 17, 600
    rng = np.random.default_rng(40 + B)
    x = np.array([int(v) for v in rng.integers(1, 1 << n, size=M)], dtype=np.uint64)
    z = np.array([int(v) for v in rng.integers(0, 1 << n, size=M)], dtype=np.uint64)
    phi = rng.uniform(-math.pi, math.pi, size=M)
    for i in range(M):
        if i % 5 == 0 or i % 37 in (1, 2, 3):
            x[i] = 0
    opts = dict(tile_qubits=B, chunk_rank=4, max_virtual=B - 4, tile_only=1)
    s = P.prx_sched_from_rotations(n, x, z, phi)
    pl = P.prx_plan_create(s, n, P.PRX_C64, 0, M, P.PRX_FUSED, opts)
    first = last = inner = 0
    for i in range(P.prx_plan_get_info(pl)["passes"]):
        ps = P.prx_plan_pass(pl, i)
        assert ps["kind"] == 2
        for c in range(ps["chunk_begin"], ps["chunk_begin"] + ps["chunk_count"]):
            ch = P.prx_plan_chunk(pl, c)
            d = [P.prx_plan_rotation(pl, ch["rot_begin"] + j)["var"] == 64
                 for j in range(ch["rot_count"])]
            first += d[0]
            last += d[-1]
            inner += any(d[j] and d[j + 1] for j in range(1, len(d) - 2))
    P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)
    assert first >= 1 and last >= 10 and inner >= 10, (first, last, inner)
    psi0 = synth.gaussian_state(n, 41)
    ref = sv.c_apply_rotations(psi0, x, z, phi)
    print(f"[diagonal records B={B}]", flush=True)
    t, info = _run_both(n, x, z, phi, psi0, P.PRX_C64, P.PRX_FUSED, opts)
    assert rel_err(to_host(t), ref) <= c64_tol(M), info


def test_empty_range_is_noop():
    n = 10
    x, z, phi = synth.random_pauli_rotations(n, 5, seed=1)
    s = P.prx_sched_from_rotations(n, x, z, phi)
    psi0 = synth.gaussian_state(n, 1)
    t = to_dev(psi0, P.PRX_C128)
    apply(t, n, P.PRX_C128, s, P.PRX_FUSED, begin=3, end=3)
    assert np.array_equal(to_host(t), psi0)
    P.prx_sched_destroy(s)


def test_resume_split_equals_single_run():
    n, M = 16, 200
    x, z, phi = synth.random_pauli_rotations(n, M, seed=21)
    s = P.prx_sched_from_rotations(n, x, z, phi)
    psi0 = synth.gaussian_state(n, 21)
    one = to_dev(psi0, P.PRX_C128)
    apply(one, n, P.PRX_C128, s, P.PRX_PLAIN)
    two = to_dev(psi0, P.PRX_C128)
    ws = workspace(P.prx_workspace_bytes(n, P.PRX_C128, s, P.PRX_PLAIN))
    P.prx_apply_range(two, n, P.PRX_C128, s, 0, 77, P.PRX_PLAIN, ws)
    P.prx_apply_range(two, n, P.PRX_C128, s, 77, M, P.PRX_PLAIN, ws)
    assert torch.equal(one, two)  # bit-identical for the plain kernel
    fused = to_dev(psi0, P.PRX_C128)
    wsf = workspace(P.prx_workspace_bytes(n, P.PRX_C128, s, P.PRX_FUSED))
    P.prx_apply_range(fused, n, P.PRX_C128, s, 0, 123, P.PRX_FUSED, wsf)
    P.prx_apply_range(fused, n, P.PRX_C128, s, 123, M, P.PRX_FUSED, wsf)
    assert rel_err(to_host(fused), to_host(one)) <= 1e-12
    P.prx_sched_destroy(s)


def test_deterministic_repeat():
    n = 18
    x, z, h = synth.jw_hamiltonian(n, 300, 2)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_trotter(H, 1, 1.0, 2, P.PRX_REORDER_SUFFIX)
    outs, ovs = [], []
    for _ in range(2):
        t = basis_state(n, synth.basis_index(n), P.PRX_C64)
        apply(t, n, P.PRX_C64, s, P.PRX_FUSED)
        outs.append(t.clone())
        ovs.append(overlap(basis_state(n, synth.basis_index(n), P.PRX_C64), t, n, P.PRX_C64))
    assert torch.equal(outs[0], outs[1]) and ovs[0] == ovs[1]
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


@pytest.mark.parametrize("n", [1, 6, 14, 21])
@pytest.mark.parametrize("dtype", [P.PRX_C128, P.PRX_C64])
def test_reductions(n, dtype):
    a = synth.gaussian_state(n, 30 + n)
    b = synth.gaussian_state(n, 60 + n)
    if dtype == P.PRX_C64:  # reference on the values the device holds
        a = a.astype(np.complex64).astype(np.complex128)
        b = b.astype(np.complex64).astype(np.complex128)
    ta, tb = to_dev(a, dtype), to_dev(b, dtype)
    ws = workspace(P.prx_reduce_workspace_bytes(n))
    ov = P.prx_overlap(ta, tb, n, dtype, ws)
    ref = sv.overlap(a, b)
    assert abs(ov - ref) <= 1e-15 * max(1.0, abs(ref))
    nn = P.prx_norm2(ta, n, dtype, ws)
    assert abs(nn - sv.norm2(a)) <= 1e-15
    k = (1 << n) - 1
    assert P.prx_amplitude(ta, n, dtype, k) == a[k]
    # a basis bra picks one amplitude
    e = basis_state(n, k // 3, dtype)
    assert P.prx_overlap(e, tb, n, dtype, ws) == b[k // 3]


def test_renormalize():
    n = 15
    a = 3.7 * synth.gaussian_state(n, 3)
    for dtype in (P.PRX_C128, P.PRX_C64):
        t = to_dev(a, dtype)
        ws = workspace(P.prx_reduce_workspace_bytes(n))
        P.prx_renormalize(t, n, dtype, ws)
        tol = 1e-14 if dtype == P.PRX_C128 else 1e-6
        assert abs(P.prx_norm2(t, n, dtype, ws) - 1.0) <= tol


def test_device_side_errors_are_reported():
    n = 10
    x, z, phi = synth.random_pauli_rotations(n, 5, seed=1)
    s = P.prx_sched_from_rotations(n, x, z, phi)
    t = to_dev(synth.gaussian_state(n, 1), P.PRX_C128)
    ws = workspace(64)
    with pytest.raises(P.PrxError) as e:
        P.prx_apply_range(t, n, P.PRX_C128, s, 0, 5, P.PRX_FUSED, ws)
    assert e.value.status == P.PRX_ERR_INVALID
    with pytest.raises(P.PrxError):
        P.prx_amplitude(t, n, P.PRX_C128, 1 << n)
    with pytest.raises(P.PrxError):
        P.prx_overlap(t, t.data_ptr() + 8, n, P.PRX_C128, workspace(1 << 20))
    P.prx_sched_destroy(s)


@pytest.mark.parametrize("dtype", [P.PRX_C128, P.PRX_C64])
def test_jw_trotter_n20_suffix_against_oracle(dtype):
    """A shortened n=20 run of the precision workload's generator (SUFFIX
    order, first order, one step of L=800) against the oracle."""
    n = 20
    x, z, h = synth.jw_hamiltonian(n, 800, 20)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_trotter(H, 1, 0.5, 1, P.PRX_REORDER_SUFFIX)
    _, rx, rz, rp = P.prx_sched_view(s)
    k0 = synth.basis_index(n)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[k0] = 1
    ref = sv.c_apply_rotations(psi0, rx, rz, rp)
    t = basis_state(n, k0, dtype)
    apply(t, n, dtype, s, P.PRX_FUSED)
    out = to_host(t)
    ov = overlap(basis_state(n, k0, dtype), t, n, dtype)
    if dtype == P.PRX_C128:
        assert rel_err(out, ref) <= 1e-12 and abs(ov - ref[k0]) <= 1e-12
    else:
        assert rel_err(out, ref) <= c64_tol(len(rx)) and abs(ov - ref[k0]) <= 1e-4
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


@pytest.mark.parametrize("dtype,kernel,opts,n", [
    # non-persistent tile kernel: 2^(16-10) = 64 tile-sets over 4 workgroups
    (P.PRX_C64, P.PRX_FUSED, dict(tile_qubits=10, chunk_rank=4, max_virtual=6, max_grid=4), 16),
    (P.PRX_C128, P.PRX_FUSED, dict(tile_qubits=11, max_virtual=7, max_grid=5), 16),
    # persistent 14-qubit tile kernel: 16 tile-sets over 3 workgroups
    (P.PRX_C64, P.PRX_FUSED, dict(tile_qubits=14, max_virtual=10, max_grid=3), 18),
    # persistent 13-qubit complex128 tile kernel: 16 tile-sets over 3 workgroups
    (P.PRX_C128, P.PRX_FUSED, dict(tile_qubits=13, max_virtual=9, max_grid=3), 17),
    # span passes only (a frame larger than the state) and the plain sweeps
    (P.PRX_C128, P.PRX_FUSED, dict(tile_qubits=15, span_max=4, max_grid=3), 14),
    (P.PRX_C64, P.PRX_PLAIN, dict(max_grid=3), 15),
    (P.PRX_C128, P.PRX_PLAIN, dict(max_grid=2), 15),
])
def test_capped_grids_stride_over_the_state(dtype, kernel, opts, n):
    """With the launch grid capped far below the work, every sweep kernel
    strides over the rest (as at n >= 33, where the work exceeds 2^22
    workgroups); the result equals the oracle's and, for complex128 (no
    renormalisation, so no change in any summation order), the uncapped
    launch's bit for bit."""
    M = 300
    x, z, phi = synth.random_pauli_rotations(n, M, seed=200 + n)
    psi0 = synth.gaussian_state(n, n + 1)
    ref = sv.c_apply_rotations(psi0, x, z, phi)
    print(f"[capped grid n={n} dtype={dtype} kernel={kernel} opts={opts}]", flush=True)
    t, info = _run_both(n, x, z, phi, psi0, dtype, kernel, opts)
    got = to_host(t)
    tol = 1e-12 if dtype == P.PRX_C128 else c64_tol(M)
    assert rel_err(got, ref) <= tol
    full = dict(opts)
    full.pop("max_grid")
    u, _ = _run_both(n, x, z, phi, psi0, dtype, kernel, full)
    if dtype == P.PRX_C128:
        assert np.array_equal(got, to_host(u))
