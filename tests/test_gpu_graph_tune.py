"""GPU tests of captured plan graphs and of the autotuner."""
import numpy as np
import pytest
import torch

import synth
from oracle import statevector as sv
from paper_2504_17881_amd import prx as P
from gpu_util import apply, basis_state, rel_err, to_host, workspace

pytestmark = pytest.mark.gpu


def test_plan_graph_replays_equal_eager():
    n = 16
    x, z, h = synth.jw_hamiltonian(n, 200, 4)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_trotter(H, 1, 1.0, 1, P.PRX_REORDER_SUFFIX)
    pl = P.prx_plan_create(s, n, P.PRX_C64, 0, 200, P.PRX_FUSED)
    ws = workspace(P.prx_plan_get_info(pl)["workspace_bytes"])
    P.prx_plan_upload(pl, ws)
    k0 = synth.basis_index(n)
    eager = basis_state(n, k0, P.PRX_C64)
    P.prx_plan_execute(pl, eager, ws)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    psi = basis_state(n, k0, P.PRX_C64)
    torch.cuda.synchronize()
    g = P.prx_plan_graph(pl, psi, ws, stream)
    for rep in range(3):
        psi.zero_()
        psi[k0] = 1.0
        torch.cuda.synchronize()
        P.prx_graph_launch(g, stream)
        stream.synchronize()
        assert torch.equal(psi, eager), rep
    P.prx_graph_destroy(g)
    P.prx_plan_destroy(pl)
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)


def test_autotune_picks_a_setting_and_auto_plan_is_exact():
    n = 20
    x, z, h = synth.jw_hamiltonian(n, 400, 20)
    H = P.prx_ham_create(n, x, z, h)
    s = P.prx_sched_trotter(H, 1, 0.5, 1, P.PRX_REORDER_SUFFIX)
    _, rx, rz, rp = P.prx_sched_view(s)
    scratch = basis_state(n, 3, P.PRX_C128)
    ws = workspace(64 << 20)
    seen = []
    best, trials = P.prx_autotune(scratch, n, P.PRX_C128, s, ws,
                                  progress=lambda o, ms: seen.append((o, ms)))
    print(f"[autotune] {trials} trials, best {best}", flush=True)
    assert trials >= 3 and P.prx_autotune_lookup(n, P.PRX_C128) == best
    # every timed setting is reported once, and the best is the fastest of them
    assert len(seen) == trials and all(ms > 0 for _, ms in seen)
    assert min(seen, key=lambda t: t[1])[0] == best
    k0 = synth.basis_index(n)
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[k0] = 1
    ref = sv.c_apply_rotations(psi0, rx, rz, rp)
    t = basis_state(n, k0, P.PRX_C128)
    info = apply(t, n, P.PRX_C128, s, P.PRX_AUTO)
    assert info["tile_qubits"] == best["tile_qubits"] or best["tile_qubits"] == 0
    assert rel_err(to_host(t), ref) <= 1e-12
    P.prx_sched_destroy(s)
    P.prx_ham_destroy(H)
