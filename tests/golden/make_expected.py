"""Writes the stored expected values of the larger parity cases.

Calls only the CPU oracle (``oracle/``) and the seeded generators
(``synth/``); nothing here touches the library or a GPU.

    python tests/golden/make_expected.py [case ...]

Cases:
  trotter1_n20   the precision workload's FP64 check at n = 20: synthetic JW
                 H (n=20, L=5000, seed 20), first-order Trotter, t = 0.5,
                 4 steps, lexicographic order, from the basis state with the
                 low 10 bits set (2*10^4 rotations).  Stores the overlap, the
                 squared norm and the 256 largest-magnitude amplitudes.
  trotter1_n28_step  the first Trotter step (rotations 0..1999) of the n = 28
                 Trotter workload (L=2000, seed 0, t = 1, 10 steps, given
                 order) from the basis state with the low 14 bits set.  Stores
                 the overlap, the squared norm and, in ``.npz``, the amplitudes
                 at 2^16 distinct indices drawn uniformly over [0, 2^28)
                 (``default_rng(28)``) plus the 4096 largest in magnitude.
  qdrift_batch   the batching workload: 256 qDRIFT samples (n_i uniform on
                 16..24, seed 7; per-size JW H with L = 500, seed 1000 + n;
                 N = 2000 draws, t = 1, sample i seeded with i) from the basis
                 state with the low floor(n/2) bits set.  Stores every
                 sample's overlap <k0|psi> and squared norm, and for the first
                 sample of each n, in ``.npz``, the amplitudes at up to 2^12
                 distinct uniform indices (``default_rng(n)``) plus the 256
                 largest.  Samples are run smallest n first and the file is
                 rewritten after each one, so an interrupted run resumes.
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


def _oracle_run(n, x, z, phi, k0):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[k0] = 1.0
    t0 = time.time()
    out = sv.c_apply_rotations(psi, x, z, phi, out=psi)
    return out, time.time() - t0


def _sample_indices(n, count, seed):
    """`count` distinct indices uniform over [0, 2^n) (all of them when
    2^n <= count), sorted."""
    N = 1 << n
    if N <= count:
        return np.arange(N, dtype=np.uint64)
    rng = np.random.default_rng(seed)
    idx = np.unique(rng.integers(0, N, size=2 * count, dtype=np.uint64))
    while idx.size < count:
        idx = np.unique(np.concatenate([idx, rng.integers(0, N, size=count, dtype=np.uint64)]))
    return np.sort(rng.permutation(idx)[:count])


def _amplitude_sample(out, n, count, top, seed):
    idx = _sample_indices(n, count, seed)
    big = np.argsort(-np.abs(out))[:top].astype(np.uint64)
    idx = np.unique(np.concatenate([idx, big]))
    vals = out[idx.astype(np.int64)]
    return idx, vals


def _run(name, n, x, z, phi, k0, meta):
    out, dt = _oracle_run(n, x, z, phi, k0)
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


def trotter1_n28_step():
    n, L, R = 28, 2000, 2000
    x, z, h = synth.jw_hamiltonian(n, L, 0)
    rx, rz, rp = S.trotter(x, z, h, 1, 1.0, 10, suffix=False)
    k0 = synth.basis_index(n)
    out, dt = _oracle_run(n, rx[:R], rz[:R], rp[:R], k0)
    idx, vals = _amplitude_sample(out, n, 1 << 16, 4096, 28)
    np.savez(os.path.join(HERE, "trotter1_n28_step.npz"), idx=idx, re=vals.real, im=vals.imag)
    rec = {
        "citation": "oracle output (scatter-form FP64 C oracle) for the first Trotter step "
                    "(rotations [0, 2000)) of the n=28 Trotter workload; generator "
                    "synth.jw_hamiltonian(28, 2000, 0), first-order Trotter t=1, 10 steps, "
                    "given order",
        "generator": "synth.jw_hamiltonian(28, 2000, 0)",
        "schedule": "trotter order=1 t=1.0 steps=10 suffix=False; rotations [0, 2000)",
        "n": n, "rotations": R, "basis_index": int(k0),
        "overlap": [float(out[k0].real), float(out[k0].imag)],
        "norm2": sv.c_norm2(out),
        "amplitudes": "trotter1_n28_step.npz: idx (2^16 uniform indices, default_rng(28), "
                      "and the 4096 largest |amplitude|), re, im",
        "oracle_seconds": round(dt, 1),
    }
    with open(os.path.join(HERE, "trotter1_n28_step.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(f"trotter1_n28_step: {R} rotations in {dt:.1f} s", flush=True)


def qdrift_batch_schedules():
    """(ns, [(x, z, phi)], basis) of the batching workload, from the oracle's
    own schedule builder."""
    w = synth.WORKLOADS["qdrift_batch"]
    ns = synth.batch_qubit_counts(w["S"], w["n_lo"], w["n_hi"], w["n_seed"])
    hams = {n: synth.jw_hamiltonian(n, w["L"], 1000 + n) for n in sorted(set(ns))}
    scheds = [S.qdrift(*hams[n], w["t"], w["N"], i) for i, n in enumerate(ns)]
    return ns, scheds, [synth.basis_index(n) for n in ns]


def qdrift_batch():
    w = synth.WORKLOADS["qdrift_batch"]
    path = os.path.join(HERE, "qdrift_batch.json")
    ns, scheds, basis = qdrift_batch_schedules()
    rec = {
        "citation": "oracle output (scatter-form FP64 C oracle) for the batching workload: "
                    "256 qDRIFT samples, n_i = synth.batch_qubit_counts(256, 16, 24, 7), "
                    "H = synth.jw_hamiltonian(n, 500, 1000 + n), N = 2000, t = 1, "
                    "sample i seeded with i, initial basis state synth.basis_index(n)",
        "S": len(ns), "N": w["N"], "t": w["t"], "L": w["L"], "n": ns,
        "overlap": [None] * len(ns), "norm2": [None] * len(ns),
        "representatives": {}, "oracle_seconds": 0.0,
    }
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
        if old.get("n") == ns:
            rec.update({k: old[k] for k in ("overlap", "norm2", "representatives",
                                            "oracle_seconds")})
    reps = {}
    for i, n in enumerate(ns):
        reps.setdefault(n, i)
    for i in sorted(range(len(ns)), key=lambda i: (ns[i], i)):
        if rec["overlap"][i] is not None:
            continue
        n = ns[i]
        x, z, phi = scheds[i]
        out, dt = _oracle_run(n, x, z, phi, basis[i])
        rec["overlap"][i] = [float(out[basis[i]].real), float(out[basis[i]].imag)]
        rec["norm2"][i] = sv.c_norm2(out)
        rec["oracle_seconds"] = round(rec["oracle_seconds"] + dt, 1)
        if reps[n] == i:
            idx, vals = _amplitude_sample(out, n, 1 << 12, 256, n)
            fname = f"qdrift_batch_n{n}.npz"
            np.savez(os.path.join(HERE, fname), idx=idx, re=vals.real, im=vals.imag)
            rec["representatives"][str(n)] = {"sample": i, "amplitudes": fname}
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        print(f"qdrift_batch: sample {i} (n={n}) in {dt:.1f} s", flush=True)


CASES = {"trotter1_n20": trotter1_n20, "trotter1_n28_step": trotter1_n28_step,
         "qdrift_batch": qdrift_batch}

if __name__ == "__main__":
    for c in (sys.argv[1:] or list(CASES)):
        CASES[c]()
