"""GPU parity at the workloads' full sizes.

Where the oracle cannot run the whole workload, the checks are (a) stored
oracle values for a prefix or a smaller instance (tests/golden, written by
tests/golden/make_expected.py from the oracle only) and (b) properties that
hold at any size: the fused kernels equal the plain kernel, complex64 equals
complex128 within the FP32 bound, and the norm is preserved.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import synth
from paper_2504_17881_amd import prx as P
from gpu_util import apply, basis_state, dev, to_host, workspace

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
EPS32 = 2.0 ** -24


def _golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)


def _check_samples(t, g, tol):
    idx = torch.tensor([s[0] for s in g["samples"]], dtype=torch.int64, device=t.device)
    got = t[idx].to(torch.complex128).cpu().numpy()
    ref = np.array([complex(s[1], s[2]) for s in g["samples"]])
    return float(np.max(np.abs(got - ref))), got, ref


def _diff_norm(a: torch.Tensor, b: torch.Tensor, chunk=1 << 27) -> float:
    """||a - b||_2 computed in FP64 chunk by chunk (no full-size temporaries)."""
    acc = 0.0
    for s in range(0, a.numel(), chunk):
        d = a[s:s + chunk].to(torch.complex128) - b[s:s + chunk].to(torch.complex128)
        acc += float(torch.sum(d.real * d.real + d.imag * d.imag))
    return math.sqrt(acc)


def _jw_sched(n, L, seed, order, t, steps, suffix):
    x, z, h = synth.jw_hamiltonian(n, L, seed)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_trotter(H, order, t, steps,
                            P.PRX_REORDER_SUFFIX if suffix else P.PRX_REORDER_NONE)
    return H, s


@pytest.mark.parametrize("dtype,kernel", [(P.PRX_C128, P.PRX_PLAIN), (P.PRX_C128, P.PRX_FUSED),
                                          (P.PRX_C64, P.PRX_FUSED)])
def test_trotter1_n20_against_stored_oracle(dtype, kernel):
    """The precision workload's FP64 check (n=20, 2*10^4 rotations)."""
    g = _golden("trotter1_n20")
    H, s = _jw_sched(20, 5000, 20, 1, 0.5, 4, True)
    t = basis_state(20, g["basis_index"], dtype)
    print(f"[n20 dtype={dtype} kernel={kernel}]", flush=True)
    apply(t, 20, dtype, s, kernel)
    err, _, _ = _check_samples(t, g, 0)
    ov = P.prx_amplitude(t, 20, dtype, g["basis_index"])
    dov = abs(ov - complex(*g["overlap"]))
    if dtype == P.PRX_C128:
        assert err <= 1e-12 and dov <= 1e-12, (err, dov)
    else:
        assert err <= 1e-4 and dov <= 1e-4, (err, dov)
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


def test_trotter1_n28_prefix_against_stored_oracle():
    g = _golden("trotter1_n28_prefix")
    H, s = _jw_sched(28, 2000, 0, 1, 1.0, 10, False)
    for kernel in (P.PRX_PLAIN, P.PRX_FUSED):
        t = basis_state(28, g["basis_index"], P.PRX_C128)
        apply(t, 28, P.PRX_C128, s, kernel, 0, g["rotations"])
        err, _, _ = _check_samples(t, g, 0)
        assert err <= 1e-12, (kernel, err)
        del t
        torch.cuda.empty_cache()
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


def test_trotter1_n28_full_fused_equals_plain():
    """The n=28 Trotter workload (2*10^4 rotations, complex128, 4 GiB): the
    fused plan equals the one-rotation-per-sweep plan element by element."""
    H, s = _jw_sched(28, 2000, 0, 1, 1.0, 10, False)
    k0 = synth.basis_index(28)
    a = basis_state(28, k0, P.PRX_C128)
    apply(a, 28, P.PRX_C128, s, P.PRX_FUSED)
    b = basis_state(28, k0, P.PRX_C128)
    apply(b, 28, P.PRX_C128, s, P.PRX_PLAIN)
    ws = workspace(P.prx_reduce_workspace_bytes(28))
    nrm = P.prx_norm2(a, 28, P.PRX_C128, ws)
    d = _diff_norm(a, b)
    oa = P.prx_amplitude(a, 28, P.PRX_C128, k0)
    ob = P.prx_amplitude(b, 28, P.PRX_C128, k0)
    print(f"[n28 full] ||fused-plain|| = {d:.3e}, |norm-1| = {abs(nrm - 1):.3e}, "
          f"overlap {oa}", flush=True)
    assert d <= 1e-12 and abs(nrm - 1.0) <= 1e-12 and abs(oa - ob) <= 1e-12
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


def test_trotter1_n32_c64_fused_against_c128_plain_prefix():
    """The precision workload at n=32: complex64 fused (32 GiB) against
    complex128 plain (64 GiB) on the first 500 rotations."""
    H, s = _jw_sched(32, 5000, 0, 1, 0.5, 4, True)
    k0 = synth.basis_index(32)
    R = 500
    a = basis_state(32, k0, P.PRX_C64)
    apply(a, 32, P.PRX_C64, s, P.PRX_FUSED, 0, R)
    b = basis_state(32, k0, P.PRX_C128)
    apply(b, 32, P.PRX_C128, s, P.PRX_PLAIN, 0, R)
    d = _diff_norm(a, b)
    oa = P.prx_amplitude(a, 32, P.PRX_C64, k0)
    ob = P.prx_amplitude(b, 32, P.PRX_C128, k0)
    print(f"[n32 prefix {R}] err_l2 = {d:.3e}, |d overlap| = {abs(oa - ob):.3e}", flush=True)
    assert d <= 8 * EPS32 * math.sqrt(R) and abs(oa - ob) <= 1e-4
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


def test_trotter1_n32_c64_tuned_launch_against_c128_plain_prefix():
    """The benchmark's own launch configuration: the committed autotune cache
    selects 14-qubit persistent tile-sets with up to 10 virtual qubits for
    n = 32 complex64 (PRX_AUTO), checked on rotations 2500..3499 of the
    benchmark schedule (the step's high-qubit terms, where the passes use
    most virtual qubits) against the complex128 one-rotation sweep."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    P.prx_autotune_load(os.path.join(root, "paper_2504_17881_amd", "tuning", "gfx950.json"))
    H, s = _jw_sched(32, 5000, 0, 1, 0.5, 4, True)
    k0 = synth.basis_index(32)
    r0, R = 2500, 1000
    a = basis_state(32, k0, P.PRX_C64)
    info = apply(a, 32, P.PRX_C64, s, P.PRX_AUTO, r0, r0 + R)
    assert info["tile_qubits"] == 14 and info["tile_passes"] == info["passes"]
    b = basis_state(32, k0, P.PRX_C128)
    apply(b, 32, P.PRX_C128, s, P.PRX_PLAIN, r0, r0 + R)
    d = _diff_norm(a, b)
    oa = P.prx_amplitude(a, 32, P.PRX_C64, k0)
    ob = P.prx_amplitude(b, 32, P.PRX_C128, k0)
    print(f"[n32 tuned prefix {R}] passes {info['passes']} err_l2 = {d:.3e}, "
          f"|d overlap| = {abs(oa - ob):.3e}", flush=True)
    assert d <= 8 * EPS32 * math.sqrt(R) and abs(oa - ob) <= 1e-4
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)
    del a, b
    torch.cuda.empty_cache()


def test_trotter1_n32_c128_tuned_launch_against_plain():
    """The committed autotune entry for n = 32 complex128 (12-qubit tile-sets,
    up to 8 virtual qubits, PRX_AUTO) against the complex128 one-rotation
    sweep on rotations 2500..2999 of the benchmark schedule (64 GiB each)."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    P.prx_autotune_load(os.path.join(root, "paper_2504_17881_amd", "tuning", "gfx950.json"))
    H, s = _jw_sched(32, 5000, 0, 1, 0.5, 4, True)
    k0 = synth.basis_index(32)
    r0, R = 2500, 500
    a = basis_state(32, k0, P.PRX_C128)
    info = apply(a, 32, P.PRX_C128, s, P.PRX_AUTO, r0, r0 + R)
    assert info["tile_qubits"] == 12 and info["tile_passes"] > 0
    d_norm = math.sqrt(P.prx_norm2(a, 32, P.PRX_C128, workspace(P.prx_reduce_workspace_bytes(32))))
    oa = P.prx_amplitude(a, 32, P.PRX_C128, k0)
    b = basis_state(32, k0, P.PRX_C128)
    apply(b, 32, P.PRX_C128, s, P.PRX_PLAIN, r0, r0 + R)
    d = _diff_norm(a, b)
    ob = P.prx_amplitude(b, 32, P.PRX_C128, k0)
    print(f"[n32 c128 tuned {R}] passes {info['passes']} err_l2 = {d:.3e}, "
          f"|d overlap| = {abs(oa - ob):.3e}", flush=True)
    assert d <= 1e-12 and abs(oa - ob) <= 1e-12 and abs(d_norm - 1.0) <= 1e-12
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)
    del a, b
    torch.cuda.empty_cache()


def _partial(n):
    x, z, h = synth.jw_hamiltonian(n, 8200, 0)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_partial(H, 200, 1.0, 5, 1000, 0, P.PRX_REORDER_SUFFIX)
    return H, s


def test_partial_n33_c64_fused_against_c128_plain_prefix():
    """Companion of the large-state workload: n=33, complex64 fused (64 GiB)
    against complex128 plain (128 GiB) on the first 300 rotations."""
    H, s = _partial(33)
    k0 = synth.basis_index(33)
    R = 300
    a = basis_state(33, k0, P.PRX_C64)
    apply(a, 33, P.PRX_C64, s, P.PRX_FUSED, 0, R, opts=dict(commuting=1))
    b = basis_state(33, k0, P.PRX_C128)
    apply(b, 33, P.PRX_C128, s, P.PRX_PLAIN, 0, R)
    d = _diff_norm(a, b)
    oa = P.prx_amplitude(a, 33, P.PRX_C64, k0)
    ob = P.prx_amplitude(b, 33, P.PRX_C128, k0)
    print(f"[n33 prefix {R}] err_l2 = {d:.3e}, |d overlap| = {abs(oa - ob):.3e}", flush=True)
    assert d <= 8 * EPS32 * math.sqrt(R) and abs(oa - ob) <= 1e-4
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


def test_partial_n34_c64_one_step():
    """The large-state workload (n=34, complex64, 128 GiB): one step of the
    partially randomised formula (200 deterministic terms twice, 1000 draws),
    fused with commuting reorders; the FP64-renormalised norm stays 1."""
    H, s = _partial(34)
    k0 = synth.basis_index(34)
    per_step = 2 * 200 + 1000
    a = basis_state(34, k0, P.PRX_C64)
    info = apply(a, 34, P.PRX_C64, s, P.PRX_FUSED, 0, per_step, opts=dict(commuting=1))
    ws = workspace(P.prx_reduce_workspace_bytes(34))
    nrm = P.prx_norm2(a, 34, P.PRX_C64, ws)
    print(f"[n34 step] passes {info['passes']} mean fuse {info['mean_fuse']:.2f} "
          f"|norm-1| {abs(nrm - 1):.2e}", flush=True)
    assert abs(nrm - 1.0) <= 1e-4
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)
