"""Writes the stored expected values of the larger parity cases.

Calls only the CPU oracle (``oracle/``) and the seeded generators
(``synth/``); nothing here touches the library or a GPU.

    python tests/golden/make_expected.py [case ...]

Cases:
  trotter1_n20   the precision workload's FP64 check at n = 20: synthetic JW
                 H (n=20, L=5000, seed 20), first-order Trotter, t = 0.5,
                 4 steps, lexicographic order, from the basis state with the
                 low 10 bits set (2*10^4 rotations).
  trotter1_n28_prefix  the first 20 rotations of the n = 28 Trotter workload
                 (L=2000, seed 0, t = 1, 10 steps, given order) from the basis
                 state with the low 14 bits set.
Each file stores the overlap with the initial basis state, the squared norm,
and the 256 largest-magnitude amplitudes (index, re, im).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import schedules as S  # noqa: E402
from oracle import statevector as sv  # noqa: E402


def _run(name, n, x, z, phi, k0, meta):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[k0] = 1.0
    t0 = time.time()
    out = sv.c_apply_rotations(psi, x, z, phi, out=psi)
    dt = time.time() - t0
    top = np.argsort(-np.abs(out))[:256]
    top.sort()
    rec = dict(meta)
    rec.update({
        "n": n, "rotations": int(len(x)), "basis_index": int(k0),
        "overlap": [float(out[k0].real), float(out[k0].imag)],
        "norm2": sv.c_norm2(out),
        "samples": [[int(k), float(out[k].real), float(out[k].imag)] for k in top],
        "oracle_seconds": round(dt, 1),
    })
    path = os.path.join(HERE, f"{name}.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"{name}: {len(x)} rotations in {dt:.1f} s -> {path}", flush=True)


def trotter1_n20():
    n, L = 20, 5000
    x, z, h = synth.jw_hamiltonian(n, L, 20)
    rx, rz, rp = S.trotter(x, z, h, 1, 0.5, 4, suffix=True)
    _run("trotter1_n20", n, rx, rz, rp, synth.basis_index(n), {
        "citation": "oracle output (scatter-form FP64 C oracle) for the n=20 check of the "
                    "precision workload; generator synth.jw_hamiltonian(20, 5000, 20), "
                    "first-order Trotter t=0.5, 4 steps, lexicographic order",
        "generator": "synth.jw_hamiltonian(20, 5000, 20)",
        "schedule": "trotter order=1 t=0.5 steps=4 suffix=True",
    })


def trotter1_n28_prefix():
    n, L = 28, 2000
    x, z, h = synth.jw_hamiltonian(n, L, 0)
    rx, rz, rp = S.trotter(x, z, h, 1, 1.0, 10, suffix=False)
    _run("trotter1_n28_prefix", n, rx[:20], rz[:20], rp[:20], synth.basis_index(n), {
        "citation": "oracle output (scatter-form FP64 C oracle) for the first 20 rotations "
                    "of the n=28 Trotter workload; generator synth.jw_hamiltonian(28, 2000, 0), "
                    "first-order Trotter t=1, 10 steps, given order",
        "generator": "synth.jw_hamiltonian(28, 2000, 0)",
        "schedule": "trotter order=1 t=1.0 steps=10 suffix=False; rotations [0, 20)",
    })


CASES = {"trotter1_n20": trotter1_n20, "trotter1_n28_prefix": trotter1_n28_prefix}

if __name__ == "__main__":
    for c in (sys.argv[1:] or list(CASES)):
        CASES[c]()
