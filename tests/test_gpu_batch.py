"""Tests of the first batched design: one persistent kernel pulling (sample,
pass, slice) items from an atomic queue, with per-sample completion counters
that later items waited on.  Its first GPU run did not complete (the test
timed out inside the kernel), and so did the one run of a revised wait loop,
so that design was switched off (removed from the library) and these tests
are skipped.  The cause was found later on the CPU, in the gfx950 code of the
same constructs: each spin iteration's acquire load invalidated its XCD's
whole L2 (buffer_inv sc1) and each finished item wrote the L2 back twice
(buffer_wbl2 sc1), which with ~1000 waiting workgroups collapses throughput,
while the iteration-count bound on a wait exceeded the test's time limit.  The batched path the library now
builds (one kernel per pass round, no cross-workgroup waits) is tested in
tests/test_gpu_batch_rounds.py.
"""
import math
import time

import numpy as np
import pytest
import torch

import synth
from oracle import schedules as S
from oracle import statevector as sv
from paper_2504_17881_amd import prx as P
from gpu_util import apply, basis_state, dev, rel_err, tdtype, to_dev, to_host, workspace

pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="queue-based persistent batch kernel with cross-workgroup waits did not finish on the GPU twice (per-iteration L2 invalidation in its spin waits); design switched off")]

EPS32 = 2.0 ** -24


def _batch_inputs(ns, L, N, t, dtype, seed0=0):
    hams, scheds, refs_in = {}, [], []
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
def test_batch_matches_oracle_per_sample(dtype):
    ns = [6, 9, 12, 7, 14, 10, 8, 13, 11, 6, 15, 9]
    hams, scheds = _batch_inputs(ns, 60, 150, 1.0, dtype)
    basis = [synth.basis_index(n) for n in ns]
    psis = [basis_state(n, b, dtype) for n, b in zip(ns, basis)]
    b = P.prx_batch_create(ns, scheds, dtype, basis)
    ws = workspace(P.prx_batch_workspace_bytes(b))
    ovd = torch.zeros(2 * len(ns), dtype=torch.float64, device=dev())
    P.prx_batch_upload(b, psis, ws)
    print(f"[batch dtype={dtype} S={len(ns)}]", flush=True)
    P.prx_batch_execute(b, ws, ovd)
    P.prx_batch_check(b, ws)
    ov = ovd.cpu().numpy()
    for i, n in enumerate(ns):
        x, z, h, _ = hams[n]
        rx, rz, rp = S.qdrift(x, z, h, 1.0, 150, i)
        psi0 = np.zeros(1 << n, dtype=np.complex128)
        psi0[basis[i]] = 1
        ref = sv.c_apply_rotations(psi0, rx, rz, rp)
        out = to_host(psis[i])
        tol = 1e-12 if dtype == P.PRX_C128 else 8 * EPS32 * math.sqrt(150) + 1e-6
        assert rel_err(out, ref) <= tol, (i, n)
        assert abs(complex(ov[2 * i], ov[2 * i + 1]) - ref[basis[i]]) <= max(tol, 1e-12)
    P.prx_batch_destroy(b)
    _free(hams, scheds)


def test_batch_run_one_call_and_replay_from_graph():
    dtype = P.PRX_C64
    ns = [8, 11, 16, 9, 12]
    hams, scheds = _batch_inputs(ns, 50, 120, 0.7, dtype, seed0=40)
    basis = [synth.basis_index(n) for n in ns]
    b = P.prx_batch_create(ns, scheds, dtype, basis)
    need = P.prx_batch_workspace_bytes(b) + 256 + 16 * len(ns)
    P.prx_batch_destroy(b)
    psis = [basis_state(n, k, dtype) for n, k in zip(ns, basis)]
    ws = workspace(need + 256)
    eager = P.prx_batch_run(psis, ns, scheds, dtype, basis, ws)
    # graph: capture once, replay three times with eager re-initialisation
    stream = torch.cuda.Stream()
    b = P.prx_batch_create(ns, scheds, dtype, basis)
    ws2 = workspace(P.prx_batch_workspace_bytes(b))
    ovd = torch.zeros(2 * len(ns), dtype=torch.float64, device=dev())
    psis2 = [basis_state(n, k, dtype) for n, k in zip(ns, basis)]
    P.prx_batch_upload(b, psis2, ws2, stream=stream)
    with torch.cuda.stream(stream):
        g = P.prx_batch_graph(b, ws2, ovd, stream)
    for rep in range(3):
        for t, k in zip(psis2, basis):
            t.zero_()
            t[k] = 1.0
        torch.cuda.synchronize()
        P.prx_graph_launch(g, stream)
        stream.synchronize()
        P.prx_batch_check(b, ws2, stream=stream)
        ov = ovd.cpu().numpy()
        got = ov[0::2] + 1j * ov[1::2]
        assert np.array_equal(got, eager), rep
    P.prx_graph_destroy(g)
    P.prx_batch_destroy(b)
    _free(hams, scheds)


def test_qdrift_batch_workload_full_size():
    """The batching workload: 256 qDRIFT samples, n uniform on {16..24}, L=500
    per-size Hamiltonians, N=2000 draws, t=1, complex64, basis states, one
    persistent launch.  Checks: every sample's norm stays 1 within the FP32
    drift bound, and the smallest samples' overlaps against the oracle."""
    w = synth.WORKLOADS["qdrift_batch"]
    ns = synth.batch_qubit_counts(w["S"], w["n_lo"], w["n_hi"], w["n_seed"])
    dtype = P.PRX_C64
    hams, scheds = _batch_inputs(ns, w["L"], w["N"], w["t"], dtype)
    basis = [synth.basis_index(n) for n in ns]
    psis = [basis_state(n, k, dtype) for n, k in zip(ns, basis)]
    b = P.prx_batch_create(ns, scheds, dtype, basis)
    ws = workspace(P.prx_batch_workspace_bytes(b))
    ovd = torch.zeros(2 * len(ns), dtype=torch.float64, device=dev())
    P.prx_batch_upload(b, psis, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.prx_batch_execute(b, ws, ovd)
    P.prx_batch_check(b, ws)
    dt = time.perf_counter() - t0
    ov = ovd.cpu().numpy()
    ovc = ov[0::2] + 1j * ov[1::2]
    print(f"[qdrift batch] S={len(ns)} {dt:.3f} s, {len(ns) / dt:.1f} samples/s, "
          f"mean overlap {np.mean(ovc):.6f}", flush=True)
    rws = workspace(P.prx_reduce_workspace_bytes(24))
    for i, n in enumerate(ns):
        nn = P.prx_norm2(psis[i], n, dtype, rws)
        assert abs(nn - 1.0) <= 1e-4, (i, n, nn)
    small = [i for i, n in enumerate(ns) if n == min(ns)][:3]
    for i in small:
        n = ns[i]
        x, z, h, _ = hams[n]
        rx, rz, rp = S.qdrift(x, z, h, w["t"], w["N"], i)
        psi0 = np.zeros(1 << n, dtype=np.complex128)
        psi0[basis[i]] = 1
        ref = sv.c_apply_rotations(psi0, rx, rz, rp)
        assert abs(ovc[i] - ref[basis[i]]) <= 1e-4
    P.prx_batch_destroy(b)
    _free(hams, scheds)


