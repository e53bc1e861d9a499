"""Planner checks on the host: the exported plan, executed by an independent
interpreter (tests/plan_interp.py), reproduces the oracle; kernel rotations
compose to the schedule; commuting reorders are legal; passes are closed."""
import math

import numpy as np
import pytest

import synth
from oracle import statevector as sv
from paper_2504_17881_amd import prx as P
from plan_interp import run_plan


def _sched(n, x, z, phi):
    return P.prx_sched_from_rotations(n, x, z, phi)


def _check_composition(plan, x, z, phi, commuting=False):
    info = P.prx_plan_get_info(plan)
    rots = [P.prx_plan_rotation(plan, i) for i in range(info["kernel_rotations"])]
    # every schedule rotation appears once, possibly as two half angles
    by_src = {}
    for r in rots:
        by_src.setdefault(r["source"], []).append(r)
    assert sorted(by_src) == list(range(len(x)))
    for j, rs in by_src.items():
        assert all(r["x"] == x[j] and r["z"] == z[j] for r in rs)
        tot = sum(r["phi"] for r in rs)
        assert abs(tot - phi[j]) <= 1e-15 * max(1.0, abs(phi[j])) * len(rs)
        if len(rs) > 1:  # equal pieces, only for large angles
            assert abs(math.tan(phi[j])) > 2 ** -0.5 and len({r["phi"] for r in rs}) == 1
        fused = info["passes"] != info["plain_passes"]
        assert all(abs(math.tan(r["phi"])) <= 2 ** -0.5 + 1e-15 or not fused for r in rs)
    order = [r["source"] for r in rots]
    if not commuting:
        assert order == sorted(order)
    else:
        # any inversion must be between commuting rotations
        for a in range(len(order)):
            for b in range(a + 1, len(order)):
                if order[a] > order[b]:
                    ra, rb = rots[a], rots[b]
                    sym = bin((ra["x"] & rb["z"]) ^ (ra["z"] & rb["x"])).count("1")
                    assert sym % 2 == 0


def _check_closure(plan, n):
    info = P.prx_plan_get_info(plan)
    for pi in range(info["passes"]):
        ps = P.prx_plan_pass(plan, pi)
        rots = [P.prx_plan_rotation(plan, i)
                for i in range(ps["rot_begin"], ps["rot_begin"] + ps["rot_count"])]
        if ps["kind"] == 1:
            basis = ps["basis"][:ps["m"]]
            for r in rots:
                assert r["x"] == 0 or r["x"] == basis[r["slot"]]
        elif ps["kind"] == 2:
            b, g = ps["b"], ps["g"]
            span = {0}
            for i in range(g):
                span |= {s ^ int(ps["vmask"][i]) for s in span}
            assert len(span) == 1 << g  # independent masks
            for r in rots:
                assert (r["x"] >> b) in span


@pytest.mark.parametrize("n,M,dtype,opts", [
    (12, 300, P.PRX_C128, None),
    (13, 300, P.PRX_C128, dict(tile_qubits=10, chunk_rank=3)),
    (12, 200, P.PRX_C64, dict(tile_qubits=11, chunk_rank=4, max_virtual=1)),
    (11, 150, P.PRX_C128, dict(span_max=5)),
])
def test_interpreter_matches_oracle_random(n, M, dtype, opts):
    x, z, phi = synth.random_pauli_rotations(n, M, seed=n + M)
    psi0 = synth.gaussian_state(n, 2)
    s = _sched(n, x, z, phi)
    pl = P.prx_plan_create(s, n, dtype, 0, M, P.PRX_FUSED, opts)
    _check_composition(pl, x, z, phi)
    _check_closure(pl, n)
    ref = sv.c_apply_rotations(psi0, x, z, phi)
    out = run_plan(pl, psi0, n)
    tol = 1e-11 if dtype == P.PRX_C128 else 5e-5
    assert np.linalg.norm(out - ref) <= tol
    P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)


@pytest.mark.parametrize("n,opts", [
    (14, None), (14, dict(max_virtual=1)), (14, dict(tile_qubits=10, chunk_rank=4)),
    (14, dict(tile_qubits=12, chunk_rank=5)), (14, dict(commuting=1)), (14, dict(max_fuse=7)),
    (16, dict(tile_qubits=10, chunk_rank=4, max_virtual=6)),
    (18, dict(tile_qubits=12, chunk_rank=4, max_virtual=6, span_max=2)),
    (16, dict(tile_qubits=13, chunk_rank=4, max_virtual=3, span_max=2)),
])
def test_interpreter_matches_oracle_jw_trotter(n, opts):
    x, z, h = synth.jw_hamiltonian(n, 300, 7)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_trotter(H, 1, 2.0, 2, P.PRX_REORDER_SUFFIX)
    _, rx, rz, rp = P.prx_sched_view(s)
    pl = P.prx_plan_create(s, n, P.PRX_C128, 0, len(rx), P.PRX_FUSED, opts)
    info = P.prx_plan_get_info(pl)
    assert info["tile_passes"] > 0
    _check_composition(pl, rx, rz, rp, commuting=bool(opts and opts.get("commuting")))
    _check_closure(pl, n)
    psi0 = synth.gaussian_state(n, 3)
    ref = sv.c_apply_rotations(psi0, rx, rz, rp)
    out = run_plan(pl, psi0, n)
    assert np.linalg.norm(out - ref) <= 1e-11
    P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


def test_interpreter_renormalised_c64_plan():
    n = 13
    x, z, h = synth.jw_hamiltonian(n, 200, 8)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_trotter(H, 1, 1.0, 2, P.PRX_REORDER_SUFFIX)
    _, rx, rz, rp = P.prx_sched_view(s)
    pl = P.prx_plan_create(s, n, P.PRX_C64, 0, len(rx), P.PRX_FUSED)
    passes = [P.prx_plan_pass(pl, i) for i in range(P.prx_plan_get_info(pl)["passes"])]
    assert any(p["norm_out"] for p in passes)
    # the hand-off links consecutive fused passes
    for a, b in zip(passes, passes[1:]):
        assert a["norm_out"] == b["renorm_in"]
    psi0 = synth.gaussian_state(n, 4)
    ref = sv.c_apply_rotations(psi0, rx, rz, rp)
    out = run_plan(pl, psi0, n)
    assert np.linalg.norm(out - ref) <= 1e-6
    P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


def test_diagonal_only_and_identity_rotations():
    n = 10
    rng = np.random.default_rng(3)
    z = rng.integers(0, 1 << n, size=40).astype(np.uint64)
    z[5] = 0
    x = np.zeros(40, dtype=np.uint64)
    phi = rng.uniform(-3, 3, size=40)
    s = _sched(n, x, z, phi)
    pl = P.prx_plan_create(s, n, P.PRX_C128, 0, 40, P.PRX_FUSED)
    psi0 = synth.gaussian_state(n, 5)
    ref = sv.c_apply_rotations(psi0, x, z, phi)
    assert np.linalg.norm(run_plan(pl, psi0, n) - ref) <= 1e-12
    P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)


def test_sub_range_plans_compose():
    n, M = 12, 120
    x, z, phi = synth.random_pauli_rotations(n, M, seed=9)
    s = _sched(n, x, z, phi)
    psi0 = synth.gaussian_state(n, 6)
    mid = 47
    a = P.prx_plan_create(s, n, P.PRX_C128, 0, mid, P.PRX_FUSED)
    b = P.prx_plan_create(s, n, P.PRX_C128, mid, M, P.PRX_FUSED)
    out = run_plan(b, run_plan(a, psi0, n), n)
    ref = sv.c_apply_rotations(psi0, x, z, phi)
    assert np.linalg.norm(out - ref) <= 1e-11
    for p in (a, b):
        P.prx_plan_destroy(p)
    P.prx_sched_destroy(s)


@pytest.mark.parametrize("dtype,bank_bits", [(P.PRX_C64, 5), (P.PRX_C128, 4)])
def test_chunk_lanes_hit_distinct_lds_banks(dtype, bank_bits):
    """Every tile chunk's coset representatives give the lanes of one LDS
    access cycle (2^bank_bits consecutive threads) distinct low index bits,
    and the cosets of all threads partition the tile-set."""
    n = 20
    x, z, h = synth.jw_hamiltonian(n, 400, 5)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_trotter(H, 1, 1.0, 1, P.PRX_REORDER_SUFFIX)
    _, rx, _, _ = P.prx_sched_view(s)
    pl = P.prx_plan_create(s, n, dtype, 0, len(rx), P.PRX_FUSED, dict(span_max=2))
    info = P.prx_plan_get_info(pl)
    checked = 0
    for pi in range(info["passes"]):
        ps = P.prx_plan_pass(pl, pi)
        if ps["kind"] != 2:
            continue
        B, m = ps["B"], ps["m"]
        for c in range(ps["chunk_begin"], ps["chunk_begin"] + ps["chunk_count"]):
            cv = P.prx_plan_chunk(pl, c)["cvec"][:B - m]
            k0 = [0] * (1 << (B - m))
            for t in range(1, 1 << (B - m)):
                low = (t & -t).bit_length() - 1
                k0[t] = k0[t & (t - 1)] ^ cv[low]
            span = {0}
            for bv in P.prx_plan_chunk(pl, c)["basis"][:m]:
                span |= {q ^ bv for q in span}
            assert len({k ^ q for k in k0 for q in span}) == 1 << B
            g = 1 << bank_bits
            for base in range(0, len(k0), g):
                assert len({k % g for k in k0[base:base + g]}) == g
            checked += 1
    assert checked > 0
    P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


@pytest.mark.parametrize("n,dtype,B,commuting", [
    (12, P.PRX_C64, 12, 1), (16, P.PRX_C64, 12, 1), (16, P.PRX_C64, 12, 0),
    (11, P.PRX_C128, 11, 1), (14, P.PRX_C128, 11, 1), (14, P.PRX_C128, 11, 0),
])
def test_tile_only_plans_of_batched_samples(n, dtype, B, commuting):
    """The form batched samples take: qDRIFT draws in random order, every pass
    a tile pass (B tile qubits, rank-4 chunks, up to 8 virtual qubits while
    16 contiguous amplitudes remain, no renormalisation, commuting rotations
    brought forward when they fit), reproducing the oracle through the
    interpreter."""
    x, z, h = synth.jw_hamiltonian(n, 80, 1000 + n)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_qdrift(H, 1.0, 400, n)
    _, rx, rz, rp = P.prx_sched_view(s)
    opts = dict(tile_qubits=B, chunk_rank=4, max_fuse=128, max_virtual=8, renorm_every=-1,
                tile_only=1, commuting=commuting)
    pl = P.prx_plan_create(s, n, dtype, 0, len(rx), P.PRX_FUSED, opts)
    info = P.prx_plan_get_info(pl)
    assert info["tile_passes"] == info["passes"] > 0
    for pi in range(info["passes"]):
        ps = P.prx_plan_pass(pl, pi)
        assert ps["g"] <= min(8, n - B, B - 4) and ps["b"] == B - ps["g"]
    _check_composition(pl, rx, rz, rp, commuting=bool(commuting))
    _check_closure(pl, n)
    psi0 = synth.gaussian_state(n, 5)
    ref = sv.c_apply_rotations(psi0, rx, rz, rp)
    out = run_plan(pl, psi0, n)
    tol = 1e-11 if dtype == P.PRX_C128 else 5e-5
    assert np.linalg.norm(out - ref) <= tol
    P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


def test_tile_only_rejects_small_states_and_plain_kernel():
    n = 10
    x, z, phi = synth.random_pauli_rotations(n, 20, seed=3)
    s = _sched(n, x, z, phi)
    for kernel, opts in [(P.PRX_FUSED, dict(tile_only=1)),
                         (P.PRX_PLAIN, dict(tile_only=1, tile_qubits=10))]:
        with pytest.raises(P.PrxError) as e:
            P.prx_plan_create(s, n, P.PRX_C64, 0, 20, kernel, opts)
        assert e.value.status == P.PRX_ERR_INVALID
    P.prx_sched_destroy(s)


def test_random_workload_exercises_every_rank4_variant():
    """The complex64 random-rotation parity workload (GPU test
    test_random_rotations_n14_c64) reaches all 64 non-diagonal static-sign
    variants of rank-4 chunks, i.e. every entry of the kernels' jump table."""
    import collections
    w = synth.WORKLOADS["random_n14"]
    n, M = w["n"], w["M"]
    x, z, phi = synth.random_pauli_rotations(n, M, seed=w["rot_seed"])
    s = _sched(n, x, z, phi)
    pl = P.prx_plan_create(s, n, P.PRX_C64, 0, M, P.PRX_FUSED)
    info = P.prx_plan_get_info(pl)
    used = collections.Counter()
    for i in range(info["kernel_rotations"]):
        r = P.prx_plan_rotation(pl, i)
        if r["static_sign"] and r["var"] < 64:
            used[r["var"]] += 1
    assert sorted(used) == list(range(64))
    P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)


def _skewed_rotations(n, M, seed, hot, extra):
    """Rotations whose X masks hold two qubits of `hot` and `extra` random
    qubits above the low four: a qubit usage that the low index bits of the
    given order do not serve."""
    rng = np.random.default_rng(seed)
    x = np.zeros(M, dtype=np.uint64)
    z = rng.integers(0, 1 << n, size=M, dtype=np.uint64)
    for i in range(M):
        m = 0
        for q in rng.choice(hot, size=2, replace=False):
            m |= 1 << int(q)
        for _ in range(extra):
            m |= 1 << int(rng.integers(4, n))
        x[i] = m
    return x, z, rng.uniform(-0.3, 0.3, size=M)


def _layouts_of(plan, n):
    """The bit order in force at every kernel rotation: index bit of each
    qubit, following the plan's relabelling passes."""
    info = P.prx_plan_get_info(plan)
    phys = list(range(n))  # phys[q] = index bit of qubit q
    at = {}
    for pi in range(info["passes"]):
        ps = P.prx_plan_pass(plan, pi)
        if ps["kind"] == 3:
            pos, dst = ps["perm_pos"], ps["perm_dst"]
            move = {pos[j]: pos[dst[j]] for j in range(12)}
            phys = [move.get(b, b) for b in phys]
            continue
        for r in range(ps["rot_begin"], ps["rot_begin"] + ps["rot_count"]):
            at[r] = list(phys)
    return at, phys


def _map(mask, phys):
    return sum(1 << phys[q] for q in range(len(phys)) if (int(mask) >> q) & 1)


@pytest.mark.parametrize("dtype,B,G", [(P.PRX_C128, 11, 7), (P.PRX_C64, 12, 8)])
def test_relabelled_plans_match_oracle(dtype, B, G):
    """Relabelling passes (kind 3) move the qubits the next rotations use into
    the low index bits.  Two phases with different hot qubits need a
    relabelling, a layout-to-layout relabelling and the final restore; the
    interpreter, which applies the exported bit moves, reproduces the
    oracle, every kernel rotation carries the schedule's masks in the bit
    order in force, and the plan ends in the original order with fewer
    passes than without relabelling."""
    n = 17
    x1, z1, p1 = _skewed_rotations(n, 500, 6, [11, 12, 14, 15], 2)
    x2, z2, p2 = _skewed_rotations(n, 500, 7, [5, 7, 13, 16], 2)
    x, z, phi = (np.concatenate([x1, x2]), np.concatenate([z1, z2]), np.concatenate([p1, p2]))
    s = _sched(n, x, z, phi)
    psi0 = synth.gaussian_state(n, 1)
    ref = sv.c_apply_rotations(psi0, x, z, phi)
    plain = P.prx_plan_create(s, n, dtype, 0, len(x), P.PRX_FUSED,
                              dict(tile_qubits=B, max_virtual=G))
    base = P.prx_plan_get_info(plain)["passes"]
    P.prx_plan_destroy(plain)
    pl = P.prx_plan_create(s, n, dtype, 0, len(x), P.PRX_FUSED,
                           dict(tile_qubits=B, max_virtual=G, relabel=1))
    info = P.prx_plan_get_info(pl)
    assert info["relabel_passes"] >= 3 and info["passes"] < base
    at, final = _layouts_of(pl, n)
    assert final == list(range(n))
    for i in range(info["kernel_rotations"]):
        r = P.prx_plan_rotation(pl, i)
        assert r["x"] == _map(x[r["source"]], at[i]) and r["z"] == _map(z[r["source"]], at[i])
    out = run_plan(pl, psi0, n)
    tol = 1e-12 if dtype == P.PRX_C128 else 8 * 2.0 ** -24 * math.sqrt(len(x))
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) <= tol
    P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)


def test_relabel_is_ignored_on_small_states_and_uniform_usage():
    n = 12
    x, z, phi = synth.random_pauli_rotations(n, 200, seed=3)
    s = _sched(n, x, z, phi)
    pl = P.prx_plan_create(s, n, P.PRX_C64, 0, 200, P.PRX_FUSED, dict(relabel=1))
    assert P.prx_plan_get_info(pl)["relabel_passes"] == 0
    P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)


@pytest.mark.parametrize("dtype,B", [(P.PRX_C64, 12), (P.PRX_C64, 14), (P.PRX_C128, 12),
                                     (P.PRX_C128, 13)])
def test_tile_passes_keep_at_least_16_contiguous_amplitudes(dtype, B):
    """Whatever virtual-qubit count is asked for, every tile pass keeps b >= 4
    low index bits (16 contiguous amplitudes per tile): the tile kernels'
    16-byte groups and chunk layouts are built for that, and a planner that
    went below it would hand the kernel a frame it was not written for."""
    n = 20
    x, z, h = synth.jw_hamiltonian(n, 300, 3)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_trotter(H, 1, 1.0, 1, P.PRX_REORDER_SUFFIX)
    _, rx, _, _ = P.prx_sched_view(s)
    seen = 0
    for mv in (10, 8, 5):
        for extra in ({}, dict(tile_only=1), dict(commuting=1)):
            opts = dict(tile_qubits=B, chunk_rank=4, max_virtual=mv, **extra)
            pl = P.prx_plan_create(s, n, dtype, 0, len(rx), P.PRX_FUSED, opts)
            for i in range(P.prx_plan_get_info(pl)["passes"]):
                ps = P.prx_plan_pass(pl, i)
                if ps["kind"] == 2:
                    assert ps["b"] >= 4 and ps["b"] + ps["g"] == B, (opts, ps["b"], ps["g"])
                    seen += 1
            P.prx_plan_destroy(pl)
    assert seen > 0
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)
