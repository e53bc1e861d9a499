"""GPU parity on the five workloads at their stated sizes and lengths.

Each test names the workload it covers.  Where the oracle finishes in the
test's time, it runs live and the whole state is compared element by
element; where it does not, the comparison uses stored oracle values
(tests/golden, written by tests/golden/make_expected.py from the oracle
only) at uniformly drawn indices plus the largest amplitudes, and
properties that hold at any size: complex64 against complex128 over the
whole schedule (amplitude 2-norm error and |overlap difference|) and the
preserved norm.

Tolerances (the FP64 oracle as reference):
  complex128: relative 2-norm error and |overlap difference| <= 1e-12;
  complex64:  relative 2-norm error <= 8 * 2^-24 * sqrt(M) for M rotations
              (a random walk of a few FP32 roundings per rotation) and
              |overlap difference| <= 1e-4 at 10^4 rotations.
"""
import json
import math
import os
import time

import numpy as np
import pytest
import torch

import synth
from oracle import schedules as S
from oracle import statevector as sv
from paper_2504_17881_amd import prx as P
from gpu_util import apply, basis_state, dev, to_host, workspace

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")
TUNE = os.path.join(ROOT, "paper_2504_17881_amd", "tuning", "gfx950.json")
EPS32 = 2.0 ** -24


def c64_bound(M):
    return 8 * EPS32 * math.sqrt(M)


@pytest.fixture(autouse=True)
def _release_device_memory():
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _diff_norm(a: torch.Tensor, b: torch.Tensor, chunk=1 << 26) -> float:
    """||a - b||_2 in FP64, chunk by chunk (no full-size temporaries)."""
    acc = 0.0
    for s in range(0, a.numel(), chunk):
        d = a[s:s + chunk].to(torch.complex128) - b[s:s + chunk].to(torch.complex128)
        acc += float(torch.sum(d.real * d.real + d.imag * d.imag))
    return math.sqrt(acc)


def _stored_amplitudes(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        meta = json.load(f)
    return meta


def _npz(fname):
    z = np.load(os.path.join(GOLDEN, fname), allow_pickle=False)
    return z["idx"].astype(np.int64), z["re"] + 1j * z["im"]


def _gather(t: torch.Tensor, idx: np.ndarray) -> np.ndarray:
    i = torch.from_numpy(idx).to(t.device)
    return t[i].to(torch.complex128).cpu().numpy()


def _jw_trotter(n, L, seed, t, steps, suffix):
    x, z, h = synth.jw_hamiltonian(n, L, seed)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_trotter(H, 1, t, steps, P.PRX_REORDER_SUFFIX if suffix else
                            P.PRX_REORDER_NONE)
    return (x, z, h), H, s


# ------------------------------------------------------------------------
# Precision workload, FP64 check at n = 20: the whole 2*10^4-rotation run,
# whole state against the live oracle.

@pytest.fixture(scope="module")
def trotter1_n20_oracle():
    n = 20
    x, z, h = synth.jw_hamiltonian(n, 5000, 20)
    rx, rz, rp = S.trotter(x, z, h, 1, 0.5, 4, suffix=True)
    k0 = synth.basis_index(n)
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[k0] = 1.0
    work = np.empty_like(psi)
    t0 = time.time()
    for q in range(4):  # one Trotter step per call, progress after each
        sv.c_apply_rotations(psi, rx[5000 * q:5000 * (q + 1)], rz[5000 * q:5000 * (q + 1)],
                             rp[5000 * q:5000 * (q + 1)], out=psi, work=work)
        print(f"[n20 oracle] step {q + 1}/4 at {time.time() - t0:.1f} s", flush=True)
    return psi, k0


@pytest.mark.parametrize("dtype,kernel", [(P.PRX_C128, P.PRX_PLAIN), (P.PRX_C128, P.PRX_FUSED),
                                          (P.PRX_C64, P.PRX_FUSED), (P.PRX_C64, P.PRX_AUTO)])
def test_trotter1_n20_whole_state_against_live_oracle(trotter1_n20_oracle, dtype, kernel):
    ref, k0 = trotter1_n20_oracle
    n = 20
    _, H, s = _jw_trotter(n, 5000, 20, 0.5, 4, True)
    t = basis_state(n, k0, dtype)
    print(f"[n20 dtype={dtype} kernel={kernel}]", flush=True)
    apply(t, n, dtype, s, kernel)
    got = to_host(t)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    dov = abs(got[k0] - ref[k0])
    print(f"[n20 dtype={dtype} kernel={kernel}] rel err {err:.3e} |d overlap| {dov:.3e}",
          flush=True)
    if dtype == P.PRX_C128:
        assert err <= 1e-12 and dov <= 1e-12
        assert float(np.max(np.abs(got - ref))) <= 1e-12
    else:
        assert err <= c64_bound(20000) and dov <= 1e-4
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


# ------------------------------------------------------------------------
# Trotter workload at n = 28 (complex128, 4 GiB): the first Trotter step
# (2000 rotations) against stored oracle amplitudes; a short prefix against
# the live oracle over the whole state.

@pytest.mark.parametrize("kernel", [P.PRX_PLAIN, P.PRX_FUSED, P.PRX_AUTO])
def test_trotter1_n28_step_against_stored_oracle(kernel):
    meta = _stored_amplitudes("trotter1_n28_step")
    idx, ref = _npz("trotter1_n28_step.npz")
    assert idx.size >= (1 << 16)
    P.prx_autotune_load(TUNE)
    _, H, s = _jw_trotter(28, 2000, 0, 1.0, 10, False)
    k0 = meta["basis_index"]
    t = basis_state(28, k0, P.PRX_C128)
    print(f"[n28 step kernel={kernel}]", flush=True)
    info = apply(t, 28, P.PRX_C128, s, kernel, 0, meta["rotations"])
    got = _gather(t, idx)
    err = float(np.max(np.abs(got - ref)))
    dov = abs(P.prx_amplitude(t, 28, P.PRX_C128, k0) - complex(*meta["overlap"]))
    nrm = P.prx_norm2(t, 28, P.PRX_C128, workspace(P.prx_reduce_workspace_bytes(28)))
    print(f"[n28 step kernel={kernel}] passes {info['passes']} max |d| {err:.3e} "
          f"|d overlap| {dov:.3e} |norm - 1| {abs(nrm - 1):.3e}", flush=True)
    assert err <= 1e-12 and dov <= 1e-12 and abs(nrm - meta["norm2"]) <= 1e-12
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


def test_trotter1_n28_prefix_whole_state_against_live_oracle():
    n, R = 28, 12
    (x, z, h), H, s = _jw_trotter(n, 2000, 0, 1.0, 10, False)
    rx, rz, rp = S.trotter(x, z, h, 1, 1.0, 10, suffix=False)
    k0 = synth.basis_index(n)
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[k0] = 1.0
    t0 = time.time()
    sv.c_apply_rotations(ref, rx[:R], rz[:R], rp[:R], out=ref)
    print(f"[n28 prefix] oracle {R} rotations in {time.time() - t0:.1f} s", flush=True)
    for kernel in (P.PRX_PLAIN, P.PRX_FUSED):
        t = basis_state(n, k0, P.PRX_C128)
        apply(t, n, P.PRX_C128, s, kernel, 0, R)
        got = to_host(t)
        err = float(np.max(np.abs(got - ref)))
        print(f"[n28 prefix kernel={kernel}] max |d| {err:.3e}", flush=True)
        assert err <= 1e-12
        del t, got
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


# ------------------------------------------------------------------------
# Precision workload at n = 32: complex64 fused in the benchmark's launch
# configuration (autotuned) against complex128 over all 2*10^4 rotations,
# both states resident (32 + 64 GiB).  The complex128 reference is the
# fused complex128 path, which the n = 20 test pins to the oracle and the
# n = 32 window test pins to the one-rotation sweep.

def test_trotter1_n32_complex64_error_over_the_whole_run():
    P.prx_autotune_load(TUNE)
    n = 32
    _, H, s = _jw_trotter(n, 5000, 0, 0.5, 4, True)
    k0 = synth.basis_index(n)
    a = basis_state(n, k0, P.PRX_C64)
    b = basis_state(n, k0, P.PRX_C128)
    rows = []
    for r0, r1 in ((0, 10000), (10000, 20000)):
        ia = apply(a, n, P.PRX_C64, s, P.PRX_AUTO, r0, r1)
        ib = apply(b, n, P.PRX_C128, s, P.PRX_AUTO, r0, r1)
        d = _diff_norm(a, b)
        oa = P.prx_amplitude(a, n, P.PRX_C64, k0)
        ob = P.prx_amplitude(b, n, P.PRX_C128, k0)
        rows.append((r1, d, abs(oa - ob)))
        print(f"[n32 whole run] rotations {r1}: err_l2 {d:.3e} |d overlap| {abs(oa - ob):.3e} "
              f"(c64 passes {ia['passes']}, c128 passes {ib['passes']})", flush=True)
    nb = P.prx_norm2(b, n, P.PRX_C128, workspace(P.prx_reduce_workspace_bytes(n)))
    assert abs(nb - 1.0) <= 1e-12
    for r1, d, dov in rows:
        assert d <= c64_bound(r1) and dov <= 1e-4, (r1, d, dov)
    del a, b
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


# ------------------------------------------------------------------------
# Batching workload: 256 qDRIFT samples (n uniform on 16..24), one captured
# graph, every sample's overlap and their mean against the stored oracle;
# one sample of every n against stored amplitudes, and the whole state of
# one sample of every n <= 20 against the live oracle.

def test_qdrift_batch_workload_against_oracle():
    with open(os.path.join(GOLDEN, "qdrift_batch.json")) as f:
        g = json.load(f)
    w = synth.WORKLOADS["qdrift_batch"]
    ns = synth.batch_qubit_counts(w["S"], w["n_lo"], w["n_hi"], w["n_seed"])
    assert g["n"] == ns and all(v is not None for v in g["overlap"])
    hams, scheds = {}, []
    for i, n in enumerate(ns):
        if n not in hams:
            x, z, h = synth.jw_hamiltonian(n, w["L"], 1000 + n)
            hams[n] = (x, z, h, P.prx_ham_create(n, x, z, h))
        scheds.append(P.prx_sched_qdrift(hams[n][3], w["t"], w["N"], i))
    basis = [synth.basis_index(n) for n in ns]
    psis = [basis_state(n, k, P.PRX_C64) for n, k in zip(ns, basis)]
    b = P.prx_batch_create(ns, scheds, P.PRX_C64, basis)
    ws = workspace(P.prx_batch_workspace_bytes(b))
    ovd = torch.zeros(2 * len(ns), dtype=torch.float64, device=dev())
    stream = torch.cuda.Stream()
    P.prx_batch_upload(b, psis, ws, stream=stream)
    gr = P.prx_batch_graph(b, ws, ovd, stream)
    print("[qdrift batch] graph launch", flush=True)
    P.prx_graph_launch(gr, stream)
    stream.synchronize()
    ov = ovd.cpu().numpy()
    got = ov[0::2] + 1j * ov[1::2]
    ref = np.array([complex(*v) for v in g["overlap"]])
    dov = np.abs(got - ref)
    print(f"[qdrift batch] max |d overlap| {dov.max():.3e}, mean overlap {got.mean():.6f} "
          f"(oracle {ref.mean():.6f})", flush=True)
    assert dov.max() <= 1e-4
    assert abs(got.mean() - ref.mean()) <= 1e-5
    rws = workspace(P.prx_reduce_workspace_bytes(24))
    for i, n in enumerate(ns):
        assert abs(P.prx_norm2(psis[i], n, P.PRX_C64, rws) - g["norm2"][i]) <= 1e-4, i
    for n_str, rep in sorted(g["representatives"].items(), key=lambda kv: int(kv[0])):
        n, i = int(n_str), rep["sample"]
        idx, vals = _npz(rep["amplitudes"])
        got_i = _gather(psis[i], idx)
        err = float(np.linalg.norm(got_i - vals) / np.linalg.norm(vals))
        print(f"[qdrift batch] sample {i} (n={n}): sampled rel err {err:.3e}", flush=True)
        assert err <= c64_bound(w["N"]), (i, n, err)
        if n <= 20:
            x, z, h, _ = hams[n]
            rx, rz, rp = S.qdrift(x, z, h, w["t"], w["N"], i)
            psi0 = np.zeros(1 << n, dtype=np.complex128)
            psi0[basis[i]] = 1.0
            full = sv.c_apply_rotations(psi0, rx, rz, rp)
            e2 = float(np.linalg.norm(to_host(psis[i]) - full) / np.linalg.norm(full))
            print(f"[qdrift batch] sample {i} (n={n}): whole-state rel err {e2:.3e}",
                  flush=True)
            assert e2 <= c64_bound(w["N"]), (i, n, e2)
    P.prx_graph_destroy(gr)
    P.prx_batch_destroy(b)
    for s in scheds:
        P.prx_sched_destroy(s)
    for v in hams.values():
        P.prx_ham_destroy(v[3])


# ------------------------------------------------------------------------
# Large-state workload: partially randomised formula, L = 8200, the 200
# largest terms by second-order Trotter (lexicographic order), 1000 qDRIFT
# draws per step, 5 steps, t = 1.  Companion at n = 33: complex64 fused
# (64 GiB) against complex128 fused (128 GiB) over the whole schedule.  At
# n = 34 (complex64, 128 GiB) the whole schedule, with the norm and the
# overlap's agreement with the n = 33 companion's scale checked.

def _partial(n):
    x, z, h = synth.jw_hamiltonian(n, 8200, 0)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_partial(H, 200, 1.0, 5, 1000, 0, P.PRX_REORDER_SUFFIX)
    return H, s


def test_partial_n33_complex64_against_complex128_whole_schedule():
    P.prx_autotune_load(TUNE)
    n = 33
    H, s = _partial(n)
    M = P.prx_sched_view(s)[1].size
    assert M == 5 * (200 + 1000 + 200)
    k0 = synth.basis_index(n)
    a = basis_state(n, k0, P.PRX_C64)
    ia = apply(a, n, P.PRX_C64, s, P.PRX_AUTO)
    b = basis_state(n, k0, P.PRX_C128)
    ib = apply(b, n, P.PRX_C128, s, P.PRX_AUTO)
    d = _diff_norm(a, b)
    oa = P.prx_amplitude(a, n, P.PRX_C64, k0)
    ob = P.prx_amplitude(b, n, P.PRX_C128, k0)
    nb = P.prx_norm2(b, n, P.PRX_C128, workspace(P.prx_reduce_workspace_bytes(n)))
    print(f"[n33 partial] {M} rotations: err_l2 {d:.3e} |d overlap| {abs(oa - ob):.3e} "
          f"overlap {ob:.6f}; passes c64 {ia['passes']} (tile {ia['tile_qubits']}), "
          f"c128 {ib['passes']} (tile {ib['tile_qubits']}); |norm - 1| {abs(nb - 1):.1e}",
          flush=True)
    assert d <= c64_bound(M) and abs(oa - ob) <= 1e-4 and abs(nb - 1.0) <= 1e-12
    del a, b
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


def test_partial_n34_complex64_whole_schedule_and_its_inverse():
    """n = 34: the whole schedule, then its inverse (the rotations in reverse
    order with negated angles, exp(-i phi P) = exp(i phi P)^-1).  The norm is
    preserved after the forward run and the state returns to the initial
    basis state within the FP32 bound for 2 M rotations; a wrong amplitude
    anywhere in either run would leave weight outside |k0>."""
    P.prx_autotune_load(TUNE)
    n = 34
    H, s = _partial(n)
    _, x, z, phi = P.prx_sched_view(s)
    M = x.size
    inv = P.prx_sched_from_rotations(n, x[::-1].copy(), z[::-1].copy(), -phi[::-1])
    k0 = synth.basis_index(n)
    a = basis_state(n, k0, P.PRX_C64)
    rws = workspace(P.prx_reduce_workspace_bytes(n))
    t0 = time.time()
    info = apply(a, n, P.PRX_C64, s, P.PRX_AUTO)
    dt = time.time() - t0
    nrm = P.prx_norm2(a, n, P.PRX_C64, rws)
    ov = P.prx_amplitude(a, n, P.PRX_C64, k0)
    print(f"[n34 partial] {M} rotations in {dt:.1f} s, {info['passes']} passes "
          f"(tile {info['tile_qubits']}, mean fuse {info['mean_fuse']:.1f}); overlap {ov:.6f} "
          f"|norm - 1| {abs(nrm - 1):.2e}", flush=True)
    assert abs(nrm - 1.0) <= 1e-4 and 0.0 < abs(ov) <= 1.0 + 1e-4
    apply(a, n, P.PRX_C64, inv, P.PRX_AUTO)
    back = P.prx_amplitude(a, n, P.PRX_C64, k0)
    nrm2 = P.prx_norm2(a, n, P.PRX_C64, rws)
    rest = math.sqrt(max(nrm2 - abs(back) ** 2, 0.0))
    print(f"[n34 partial] after the inverse: <k0|psi> = {back:.8f}, weight elsewhere "
          f"{rest:.3e}", flush=True)
    assert abs(back - 1.0) <= c64_bound(2 * M) and rest <= c64_bound(2 * M)
    del a
    P.prx_sched_destroy(inv)
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)
