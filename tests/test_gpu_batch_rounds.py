"""GPU tests of the batched path: per pass round, one kernel over the tile-set
items of the samples planned into tile passes and one over the coset slices
of the smaller samples (no cross-workgroup waits), captured as one graph."""
import math
import time

import numpy as np
import pytest
import torch

import synth
from oracle import schedules as S
from oracle import statevector as sv
from paper_2504_17881_amd import prx as P
from gpu_util import basis_state, dev, rel_err, to_host, workspace

pytestmark = pytest.mark.gpu

EPS32 = 2.0 ** -24


def _inputs(ns, L, N, t, seed0=0):
    hams, scheds = {}, []
    for i, n in enumerate(ns):
        if n not in hams:
            x, z, h = synth.jw_hamiltonian(n, L, 1000 + n)
            hams[n] = (x, z, h, P.prx_ham_create(n, x, z, h))
        scheds.append(P.prx_sched_qdrift(hams[n][3], t, N, seed0 + i))
    return hams, scheds


def _free(hams, scheds):
    for s in scheds:
        P.prx_sched_destroy(s)
    for v in hams.values():
        P.prx_ham_destroy(v[3])


@pytest.mark.parametrize("dtype", [P.PRX_C128, P.PRX_C64])
def test_rounds_match_oracle_per_sample(dtype):
    ns = [6, 9, 12, 7, 14, 10, 8, 13, 11, 6, 15, 9]
    N = 150
    hams, scheds = _inputs(ns, 60, N, 1.0)
    basis = [synth.basis_index(n) for n in ns]
    psis = [basis_state(n, b, dtype) for n, b in zip(ns, basis)]
    b = P.prx_batch_create(ns, scheds, dtype, basis)
    ws = workspace(P.prx_batch_workspace_bytes(b))
    ovd = torch.zeros(2 * len(ns), dtype=torch.float64, device=dev())
    P.prx_batch_upload(b, psis, ws)
    print(f"[rounds dtype={dtype}] launching", flush=True)
    P.prx_batch_execute(b, ws, ovd)
    P.prx_batch_check(b, ws)
    print(f"[rounds dtype={dtype}] done", flush=True)
    ov = ovd.cpu().numpy()
    tol = 1e-12 if dtype == P.PRX_C128 else 8 * EPS32 * math.sqrt(N) + 1e-6
    for i, n in enumerate(ns):
        x, z, h, _ = hams[n]
        rx, rz, rp = S.qdrift(x, z, h, 1.0, N, i)
        psi0 = np.zeros(1 << n, dtype=np.complex128)
        psi0[basis[i]] = 1
        ref = sv.c_apply_rotations(psi0, rx, rz, rp)
        assert rel_err(to_host(psis[i]), ref) <= tol, (i, n)
        assert abs(complex(ov[2 * i], ov[2 * i + 1]) - ref[basis[i]]) <= max(tol, 1e-12)
    P.prx_batch_destroy(b)
    _free(hams, scheds)


@pytest.mark.parametrize("dtype", [P.PRX_C64, P.PRX_C128])
def test_tile_rounds_with_many_virtual_qubits(dtype):
    """Larger samples (tile passes with up to 8 virtual qubits at complex64, 7
    at complex128) of uneven pass counts next to span samples, checked
    element by element against the oracle."""
    ns = [13, 17, 20, 10, 18, 11]
    N = 500
    hams, scheds = _inputs(ns, 120, N, 0.8, seed0=77)
    basis = [synth.basis_index(n) for n in ns]
    psis = [basis_state(n, b, dtype) for n, b in zip(ns, basis)]
    b = P.prx_batch_create(ns, scheds, dtype, basis)
    info = P.prx_batch_get_info(b)
    assert info["tile_samples"] == sum(n >= (12 if dtype == P.PRX_C64 else 11) for n in ns)
    ws = workspace(P.prx_batch_workspace_bytes(b))
    ovd = torch.zeros(2 * len(ns), dtype=torch.float64, device=dev())
    P.prx_batch_upload(b, psis, ws)
    print(f"[tile rounds dtype={dtype}] rounds={info['rounds']} launching", flush=True)
    P.prx_batch_execute(b, ws, ovd)
    P.prx_batch_check(b, ws)
    print(f"[tile rounds dtype={dtype}] done", flush=True)
    ov = ovd.cpu().numpy()
    tol = 1e-12 if dtype == P.PRX_C128 else 8 * EPS32 * math.sqrt(N) + 1e-6
    for i, n in enumerate(ns):
        x, z, h, _ = hams[n]
        rx, rz, rp = S.qdrift(x, z, h, 0.8, N, 77 + i)
        psi0 = np.zeros(1 << n, dtype=np.complex128)
        psi0[basis[i]] = 1
        ref = sv.c_apply_rotations(psi0, rx, rz, rp)
        assert rel_err(to_host(psis[i]), ref) <= tol, (i, n)
        assert abs(complex(ov[2 * i], ov[2 * i + 1]) - ref[basis[i]]) <= max(tol, 1e-12)
    P.prx_batch_destroy(b)
    _free(hams, scheds)


@pytest.mark.parametrize("dtype", [P.PRX_C64, P.PRX_C128])
def test_tile_rounds_with_diagonal_terms(dtype):
    """Hamiltonians with Z-only terms: the qDRIFT draws put diagonal
    rotations inside the tile rounds' chunks (at complex64 the threaded
    rotation loop stops at each one and resumes after it)."""
    ns = [13, 16, 12]
    N = 400
    hams, scheds = {}, []
    rng = np.random.default_rng(61)
    for i, n in enumerate(ns):
        x, z, h = synth.jw_hamiltonian(n, 100, 500 + n)
        zs = set()
        while len(zs) < 40:
            zs.add(int(rng.integers(1, 1 << n)))
        x = np.concatenate([np.asarray(x, dtype=np.uint64), np.zeros(40, dtype=np.uint64)])
        z = np.concatenate([np.asarray(z, dtype=np.uint64), np.array(sorted(zs), dtype=np.uint64)])
        h = np.concatenate([np.asarray(h, dtype=np.float64), rng.normal(0.0, 0.5, size=40)])
        hams[n] = (x, z, h, P.prx_ham_create(n, x, z, h))
        scheds.append(P.prx_sched_qdrift(hams[n][3], 0.7, N, 90 + i))
    basis = [synth.basis_index(n) for n in ns]
    psis = [basis_state(n, b0, dtype) for n, b0 in zip(ns, basis)]
    b = P.prx_batch_create(ns, scheds, dtype, basis)
    assert P.prx_batch_get_info(b)["tile_samples"] == len(ns)
    ws = workspace(P.prx_batch_workspace_bytes(b))
    ovd = torch.zeros(2 * len(ns), dtype=torch.float64, device=dev())
    P.prx_batch_upload(b, psis, ws)
    print(f"[diagonal terms dtype={dtype}] launching", flush=True)
    P.prx_batch_execute(b, ws, ovd)
    P.prx_batch_check(b, ws)
    print(f"[diagonal terms dtype={dtype}] done", flush=True)
    tol = 1e-12 if dtype == P.PRX_C128 else 8 * EPS32 * math.sqrt(N) + 1e-6
    ndiag = 0
    for i, n in enumerate(ns):
        x, z, h, _ = hams[n]
        rx, rz, rp = S.qdrift(x, z, h, 0.7, N, 90 + i)
        ndiag += int(np.sum(np.asarray(rx) == 0))
        psi0 = np.zeros(1 << n, dtype=np.complex128)
        psi0[basis[i]] = 1
        ref = sv.c_apply_rotations(psi0, rx, rz, rp)
        assert rel_err(to_host(psis[i]), ref) <= tol, (i, n)
    assert ndiag >= 30
    P.prx_batch_destroy(b)
    _free(hams, scheds)


@pytest.mark.parametrize("dtype", [P.PRX_C128, P.PRX_C64])
def test_capped_round_grids_stride_over_the_items(dtype):
    """With every round launch capped at 3 workgroups, both round kernels
    stride over their items (the tile rounds hold several tile-sets per
    workgroup in turn); the states equal the oracle's and, for complex128,
    the uncapped launch's bit for bit."""
    ns = [14, 9, 13, 7, 12, 11]
    N = 200
    hams, scheds = _inputs(ns, 80, N, 0.9, seed0=300)
    basis = [synth.basis_index(n) for n in ns]
    runs = []
    for cap in (3, 0):
        psis = [basis_state(n, b0, dtype) for n, b0 in zip(ns, basis)]
        b = P.prx_batch_create(ns, scheds, dtype, basis)
        P.prx_batch_set_max_grid(b, cap)
        ws = workspace(P.prx_batch_workspace_bytes(b))
        ovd = torch.zeros(2 * len(ns), dtype=torch.float64, device=dev())
        P.prx_batch_upload(b, psis, ws)
        print(f"[capped rounds dtype={dtype} cap={cap}] launching", flush=True)
        P.prx_batch_execute(b, ws, ovd)
        P.prx_batch_check(b, ws)
        print(f"[capped rounds dtype={dtype} cap={cap}] done", flush=True)
        runs.append(([to_host(p) for p in psis], ovd.cpu().numpy()))
        P.prx_batch_destroy(b)
    tol = 1e-12 if dtype == P.PRX_C128 else 8 * EPS32 * math.sqrt(N) + 1e-6
    (capped, ovc), (full, ovf) = runs
    for i, n in enumerate(ns):
        x, z, h, _ = hams[n]
        rx, rz, rp = S.qdrift(x, z, h, 0.9, N, 300 + i)
        psi0 = np.zeros(1 << n, dtype=np.complex128)
        psi0[basis[i]] = 1
        ref = sv.c_apply_rotations(psi0, rx, rz, rp)
        assert rel_err(capped[i], ref) <= tol, (i, n)
        if dtype == P.PRX_C128:
            assert np.array_equal(capped[i], full[i]), (i, n)
    if dtype == P.PRX_C128:
        assert np.array_equal(ovc, ovf)
    _free(hams, scheds)


def _empty_sched(n):
    e = np.array([], dtype=np.uint64)
    return P.prx_sched_from_rotations(n, e, e, np.array([], dtype=np.float64))


def test_rounds_with_empty_schedules():
    """Samples with no rotations stay untouched next to a tile sample and a
    span sample; a batch of empty samples only reads the overlaps."""
    dtype = P.PRX_C64
    ns = [14, 13, 9, 8]
    N = 80
    x13, z13, h13 = synth.jw_hamiltonian(13, 40, 1013)
    x9, z9, h9 = synth.jw_hamiltonian(9, 40, 1009)
    H13 = P.prx_ham_create(13, x13, z13, h13)
    H9 = P.prx_ham_create(9, x9, z9, h9)
    scheds = [_empty_sched(14), P.prx_sched_qdrift(H13, 0.6, N, 5),
              P.prx_sched_qdrift(H9, 0.6, N, 6), _empty_sched(8)]
    basis = [synth.basis_index(n) for n in ns]
    psis = [basis_state(n, k, dtype) for n, k in zip(ns, basis)]
    b = P.prx_batch_create(ns, scheds, dtype, basis)
    info = P.prx_batch_get_info(b)
    assert info["tile_samples"] == 2 and info["rounds"] > 0
    ws = workspace(P.prx_batch_workspace_bytes(b))
    ovd = torch.zeros(2 * len(ns), dtype=torch.float64, device=dev())
    P.prx_batch_upload(b, psis, ws)
    print(f"[empty samples] rounds={info['rounds']} launching", flush=True)
    P.prx_batch_execute(b, ws, ovd)
    P.prx_batch_check(b, ws)
    print("[empty samples] done", flush=True)
    ov = ovd.cpu().numpy()
    tol = 8 * EPS32 * math.sqrt(N) + 1e-6
    for i, (n, (x, z, h), seed) in [(1, (13, (x13, z13, h13), 5)), (2, (9, (x9, z9, h9), 6))]:
        rx, rz, rp = S.qdrift(x, z, h, 0.6, N, seed)
        psi0 = np.zeros(1 << n, dtype=np.complex128)
        psi0[basis[i]] = 1
        ref = sv.c_apply_rotations(psi0, rx, rz, rp)
        assert rel_err(to_host(psis[i]), ref) <= tol, (i, n)
    for i in (0, 3):
        out = to_host(psis[i])
        assert out[basis[i]] == 1 and np.count_nonzero(out) == 1
        assert ov[2 * i] == 1.0 and ov[2 * i + 1] == 0.0
    P.prx_batch_destroy(b)
    # only empty samples: no round kernels, the overlaps still arrive
    e_scheds = [_empty_sched(14), _empty_sched(8)]
    e_ns, e_basis = [14, 8], [basis[0], basis[3]]
    e_psis = [basis_state(n, k, dtype) for n, k in zip(e_ns, e_basis)]
    b = P.prx_batch_create(e_ns, e_scheds, dtype, e_basis)
    assert P.prx_batch_get_info(b)["rounds"] == 0
    ws = workspace(P.prx_batch_workspace_bytes(b))
    ovd = torch.zeros(4, dtype=torch.float64, device=dev())
    P.prx_batch_upload(b, e_psis, ws)
    P.prx_batch_execute(b, ws, ovd)
    P.prx_batch_check(b, ws)
    assert ovd.cpu().numpy().tolist() == [1.0, 0.0, 1.0, 0.0]
    P.prx_batch_destroy(b)
    for sc in scheds + e_scheds:
        P.prx_sched_destroy(sc)
    P.prx_ham_destroy(H13)
    P.prx_ham_destroy(H9)


def test_rounds_one_call_and_graph_replay():
    dtype = P.PRX_C64
    ns = [8, 11, 16, 9, 12]
    hams, scheds = _inputs(ns, 50, 120, 0.7, seed0=40)
    basis = [synth.basis_index(n) for n in ns]
    b = P.prx_batch_create(ns, scheds, dtype, basis)
    need = P.prx_batch_workspace_bytes(b) + 256 + 16 * len(ns)
    P.prx_batch_destroy(b)
    psis = [basis_state(n, k, dtype) for n, k in zip(ns, basis)]
    eager = P.prx_batch_run(psis, ns, scheds, dtype, basis, workspace(need + 256))
    stream = torch.cuda.Stream()
    b = P.prx_batch_create(ns, scheds, dtype, basis)
    ws2 = workspace(P.prx_batch_workspace_bytes(b))
    ovd = torch.zeros(2 * len(ns), dtype=torch.float64, device=dev())
    psis2 = [basis_state(n, k, dtype) for n, k in zip(ns, basis)]
    P.prx_batch_upload(b, psis2, ws2, stream=stream)
    g = P.prx_batch_graph(b, ws2, ovd, stream)
    for rep in range(3):
        for t, k in zip(psis2, basis):
            t.zero_()
            t[k] = 1.0
        torch.cuda.synchronize()
        P.prx_graph_launch(g, stream)
        stream.synchronize()
        ov = ovd.cpu().numpy()
        assert np.array_equal(ov[0::2] + 1j * ov[1::2], eager), rep
    P.prx_graph_destroy(g)
    P.prx_batch_destroy(b)
    _free(hams, scheds)


def test_qdrift_batch_workload_full_size():
    """The batching workload: 256 qDRIFT samples, n uniform on {16..24}, per-size
    JW H with L=500, N=2000 draws, t=1, complex64, basis states, one graph
    launch.  Every sample's norm stays 1 within the FP32 bound; the smallest
    samples' overlaps match the oracle."""
    w = synth.WORKLOADS["qdrift_batch"]
    ns = synth.batch_qubit_counts(w["S"], w["n_lo"], w["n_hi"], w["n_seed"])
    dtype = P.PRX_C64
    hams, scheds = _inputs(ns, w["L"], w["N"], w["t"])
    basis = [synth.basis_index(n) for n in ns]
    psis = [basis_state(n, k, dtype) for n, k in zip(ns, basis)]
    b = P.prx_batch_create(ns, scheds, dtype, basis)
    ws = workspace(P.prx_batch_workspace_bytes(b))
    ovd = torch.zeros(2 * len(ns), dtype=torch.float64, device=dev())
    stream = torch.cuda.Stream()
    P.prx_batch_upload(b, psis, ws, stream=stream)
    g = P.prx_batch_graph(b, ws, ovd, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.prx_graph_launch(g, stream)
    stream.synchronize()
    dt = time.perf_counter() - t0
    ov = ovd.cpu().numpy()
    ovc = ov[0::2] + 1j * ov[1::2]
    print(f"[qdrift batch] S={len(ns)} {dt:.3f} s, {len(ns) / dt:.1f} samples/s, "
          f"mean overlap {np.mean(ovc):.6f}", flush=True)
    rws = workspace(P.prx_reduce_workspace_bytes(24))
    for i, n in enumerate(ns):
        nn = P.prx_norm2(psis[i], n, dtype, rws)
        assert abs(nn - 1.0) <= 1e-4, (i, n, nn)
    for i in [i for i, n in enumerate(ns) if n == min(ns)][:3]:
        n = ns[i]
        x, z, h, _ = hams[n]
        rx, rz, rp = S.qdrift(x, z, h, w["t"], w["N"], i)
        psi0 = np.zeros(1 << n, dtype=np.complex128)
        psi0[basis[i]] = 1
        ref = sv.c_apply_rotations(psi0, rx, rz, rp)
        assert abs(ovc[i] - ref[basis[i]]) <= 1e-4
    P.prx_graph_destroy(g)
    P.prx_batch_destroy(b)
    _free(hams, scheds)
