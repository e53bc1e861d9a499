"""Qubit-relabelling passes on the GPU: the permutation kernel and the
relabelled fused plans against the oracle.

A relabelling pass moves index bits in place (every 2^12-element group is
closed under the move); the rotations after it run with their masks in the
new bit order, and the plan's last pass restores the original order, so the
result is the plain rotation product, compared element by element with the
FP64 oracle: complex128 at 1e-12 (relative 2-norm), complex64 within
8 * 2^-24 * sqrt(M).
"""
import math
import time

import numpy as np
import pytest

import synth
from oracle import schedules as S
from oracle import statevector as sv
from paper_2504_17881_amd import prx as P
from gpu_util import apply, basis_state, rel_err, to_dev, to_host
from test_planner import _skewed_rotations

pytestmark = pytest.mark.gpu


def _tol(dtype, M):
    return 1e-12 if dtype == P.PRX_C128 else 8 * 2.0 ** -24 * math.sqrt(M)


@pytest.mark.parametrize("n,dtype,B,G", [(17, P.PRX_C128, 11, 7), (17, P.PRX_C64, 12, 8),
                                         (20, P.PRX_C64, 14, 10), (20, P.PRX_C128, 12, 8)])
def test_relabelled_plan_against_oracle(n, dtype, B, G):
    hot1 = [n - 6, n - 5, n - 3, n - 2]
    hot2 = [5, 7, n - 4, n - 1]
    x1, z1, p1 = _skewed_rotations(n, 500, 6, hot1, 2)
    x2, z2, p2 = _skewed_rotations(n, 500, 7, hot2, 2)
    x, z, phi = (np.concatenate([x1, x2]), np.concatenate([z1, z2]), np.concatenate([p1, p2]))
    s = P.prx_sched_from_rotations(n, x, z, phi)
    psi0 = synth.gaussian_state(n, 2)
    ref = sv.c_apply_rotations(psi0, x, z, phi)
    t = to_dev(psi0, dtype)
    print(f"[relabel n={n} dtype={dtype} B={B}]", flush=True)
    info = apply(t, n, dtype, s, P.PRX_FUSED, opts=dict(tile_qubits=B, max_virtual=G, relabel=1))
    err = rel_err(to_host(t), ref)
    print(f"[relabel n={n} dtype={dtype} B={B}] passes {info['passes']} relabelling "
          f"{info['relabel_passes']} rel err {err:.2e}", flush=True)
    assert info["relabel_passes"] >= 2
    assert err <= _tol(dtype, len(x))
    P.prx_sched_destroy(s)


def test_relabelled_qdrift_n24_against_live_oracle():
    """A qDRIFT sample of the batching workload's n = 24 Hamiltonian (2000
    draws), single state, 14-qubit tile-sets with relabelling: whole state
    against the oracle."""
    n = 24
    x, z, h = synth.jw_hamiltonian(n, 500, 1000 + n)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_qdrift(H, 1.0, 2000, 3)
    rx, rz, rp = S.qdrift(x, z, h, 1.0, 2000, 3)
    k0 = synth.basis_index(n)
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[k0] = 1.0
    t0 = time.time()
    sv.c_apply_rotations(ref, rx, rz, rp, out=ref)
    print(f"[relabel qdrift n=24] oracle {time.time() - t0:.1f} s", flush=True)
    for dtype in (P.PRX_C64, P.PRX_C128):
        B, G = (14, 10) if dtype == P.PRX_C64 else (12, 8)
        res = {}
        for rl in (0, 1):
            t = basis_state(n, k0, dtype)
            info = apply(t, n, dtype, s, P.PRX_FUSED,
                         opts=dict(tile_qubits=B, max_virtual=G, relabel=rl))
            err = rel_err(to_host(t), ref)
            res[rl] = (info["passes"], info["relabel_passes"])
            print(f"[relabel qdrift n=24 dtype={dtype}] relabel={rl} passes {info['passes']} "
                  f"(relabelling {info['relabel_passes']}) rel err {err:.2e}", flush=True)
            assert err <= _tol(dtype, 2000)
        assert res[1][1] >= 1 and res[1][0] < res[0][0]
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)
