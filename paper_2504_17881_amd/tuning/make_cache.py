"""Writes entries of the autotune cache ``gfx950.json`` on one MI355X.

    python paper_2504_17881_amd/tuning/make_cache.py [key ...] [--out PATH]

Each key is a workload and a state precision; its cache entry is keyed by
(n, dtype).  The autotuner (``prx_autotune``) times its staged search on the
first rotations of the workload's schedule (``SLICES``) applied to a basis
state, and the fastest setting is merged into the existing cache file.
Keys:
  trotter1_n28/c128   n = 28, L = 2000 JW H (seed 0), first-order Trotter,
                      t = 1, 10 steps, given order; one step timed
  trotter1_n32/c64, trotter1_n32/c128
                      n = 32, L = 5000 (seed 0), t = 0.5, 4 steps,
                      lexicographic order; one step timed
  partial_n33/c64, partial_n33/c128, partial_n34/c64
                      partially randomised formula, L = 8200 (seed 0), the
                      200 largest terms at second order, 1000 draws per step,
                      5 steps, t = 1; the first 700 rotations timed (the
                      deterministic half-step and half of the random part)
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SLICES = {"trotter1_n28": 2000, "trotter1_n32": 5000, "partial_n33": 700, "partial_n34": 700}


def schedule(P, synth, name):
    """(n, ham, sched) of a workload key's schedule."""
    if name == "trotter1_n28":
        n = 28
        x, z, h = synth.jw_hamiltonian(n, 2000, 0)
        H = P.prx_ham_create(n, x, z, h)
        return n, H, P.prx_sched_trotter(H, 1, 1.0, 10, P.PRX_REORDER_NONE)
    if name == "trotter1_n32":
        n = 32
        x, z, h = synth.jw_hamiltonian(n, 5000, 0)
        H = P.prx_ham_create(n, x, z, h)
        return n, H, P.prx_sched_trotter(H, 1, 0.5, 4, P.PRX_REORDER_SUFFIX)
    if name in ("partial_n33", "partial_n34"):
        n = int(name[-2:])
        x, z, h = synth.jw_hamiltonian(n, 8200, 0)
        H = P.prx_ham_create(n, x, z, h)
        return n, H, P.prx_sched_partial(H, 200, 1.0, 5, 1000, 0, P.PRX_REORDER_SUFFIX)
    raise KeyError(name)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("keys", nargs="*", default=["trotter1_n28/c128", "partial_n33/c64",
                                                 "partial_n33/c128", "partial_n34/c64"])
    ap.add_argument("--out", default=os.path.join(HERE, "gfx950.json"))
    args = ap.parse_args()
    import torch
    import synth
    from paper_2504_17881_amd import prx as P

    if os.path.exists(args.out):
        P.prx_autotune_load(args.out)
    dev = torch.device("cuda:0")
    ws = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    for key in args.keys:
        name, dt = key.split("/")
        dtype = P.PRX_C64 if dt == "c64" else P.PRX_C128
        n, H, s = schedule(P, synth, name)
        _, x, z, phi = P.prx_sched_view(s)
        R = min(SLICES[name], x.size)
        sub = P.prx_sched_from_rotations(n, x[:R], z[:R], phi[:R])
        psi = torch.zeros(1 << n, dtype=torch.complex64 if dtype == P.PRX_C64 else
                          torch.complex128, device=dev)
        psi[synth.basis_index(n)] = 1.0
        t0 = time.time()

        def trial(o, ms):
            print(f"[tune {key}] {({k: v for k, v in o.items() if v})} {ms:.1f} ms",
                  flush=True)
        best, trials = P.prx_autotune(psi, n, dtype, sub, ws, progress=trial)
        print(f"[tune {key}] {trials} settings in {time.time() - t0:.0f} s, best "
              f"{({k: v for k, v in best.items() if v})}", flush=True)
        P.prx_autotune_save(args.out)
        P.prx_sched_destroy(sub)
        P.prx_sched_destroy(s)
        P.prx_ham_destroy(H)
        del psi
        torch.cuda.empty_cache()
    return 0


if __name__ == "__main__":
    sys.exit(main())
