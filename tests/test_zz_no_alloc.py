"""The allocation-free entry point prx_apply_range_static against
prx_apply_range (caller workspace), through the C ABI.

Both run the same plan with the same kernels, so the results must agree
bit for bit; two calls in a row (the second on a smaller state and a
shorter range) check that the shared static buffer carries nothing from one
call into the next.  The size limit is checked on the host, before any
device work.
"""
import numpy as np
import pytest
import torch

import synth
from paper_2504_17881_amd import prx as P
from gpu_util import to_dev, to_host, workspace


def test_static_workspace_limit_is_rejected_before_device_work():
    n, M = 12, 2_200_000  # 32-byte records: above the 64 MiB buffer
    rng = np.random.default_rng(5)
    x = rng.integers(0, 4, size=M, dtype=np.uint64)
    z = rng.integers(0, 4, size=M, dtype=np.uint64)
    phi = rng.uniform(-0.1, 0.1, size=M)
    s = P.prx_sched_from_rotations(n, x, z, phi)
    with pytest.raises(P.PrxError, match="exceeds the static buffer"):
        # an address that is never dereferenced: the check precedes device work
        P.prx_apply_range_static(256, n, P.PRX_C64, s, 0, M, P.PRX_FUSED)
    P.prx_sched_destroy(s)


def _case(n, M, seed, dtype, kernel, begin, end):
    x, z, phi = synth.random_pauli_rotations(n, M, seed=seed)
    s = P.prx_sched_from_rotations(n, x, z, phi)
    psi0 = synth.gaussian_state(n, seed)
    ref = to_dev(psi0, dtype)
    ws = workspace(P.prx_workspace_bytes(n, dtype, s, kernel))
    P.prx_apply_range(ref, n, dtype, s, begin, end, kernel, ws)
    got = to_dev(psi0, dtype)
    print(f"[no-alloc] n={n} M={M} range=[{begin},{end}) dtype={dtype} kernel={kernel}",
          flush=True)
    P.prx_apply_range_static(got, n, dtype, s, begin, end, kernel)
    a, b = to_host(got), to_host(ref)
    P.prx_sched_destroy(s)
    return a, b


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [P.PRX_C64, P.PRX_C128])
def test_static_entry_point_equals_caller_workspace_twice(dtype):
    # first call: 20 qubits, 600 rotations, fused (tile passes with norm
    # partials and renormalisation for complex64)
    a, b = _case(20, 600, 11, dtype, P.PRX_FUSED, 0, 600)
    assert np.array_equal(a, b), float(np.max(np.abs(a - b)))
    assert np.linalg.norm(a - to_host(to_dev(synth.gaussian_state(20, 11), dtype))) > 0.1
    # second call, smaller: 14 qubits, a sub-range of a shorter list
    a, b = _case(14, 200, 12, dtype, P.PRX_AUTO, 17, 150)
    assert np.array_equal(a, b), float(np.max(np.abs(a - b)))
    torch.cuda.synchronize()
