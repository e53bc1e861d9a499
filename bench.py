#!/usr/bin/env python3
"""Benchmark: amplitude updates/s and HBM roofline at n=32, FP32 fused vs FP64 plain.

Workload (precision workload): synthetic Jordan-Wigner-shaped Hamiltonian,
n = 32, L = 5000 terms (seed 0), lexicographically ordered terms,
first-order Trotter with t = 0.5 and 4 steps (2*10^4 rotations), initial
basis state with the low 16 bits set.  Every Trotter step is the same
5000-rotation product, so one plan serves all steps.  A bench step is one
Trotter step applied by the fused complex64 path with FP64 renormalisation,
followed by the overlap with the initial basis state; the timed loop applies
K consecutive steps to one state (steps 1-4 are the workload's run, later
steps continue it).

Reported:
  value        amplitude updates per second of the timed steps
               (updates = rotations * 2^n; inputs resident in HBM);
  roofline     the dominant kernel (largest share of the timed steps'
               kernel time): algorithmic bytes per launch (2 * 2^n * 8 B,
               one read and one write of the state) over its average
               launch duration from HIP events recorded around every pass;
  precision    outside the timed region: the whole 4-step run in complex64
               (fused) and in complex128 (fused, tuned), both resident;
               amplitude 2-norm error and |overlap difference| of complex64
               against complex128 after 10^4 rotations and at the end, and
               the complex128 run's own rate and roofline;
  fp64_plain   the complex128 single-rotation sweep on the same schedule
               (first `--plain-rotations` rotations), for the 2x comparison;
  cpu_baseline the FP64 CPU oracle on the first rotations of the same
               schedule and state on all host cores, plus one core and the
               n = 28 Trotter workload's 100-rotation rate.

    python bench.py [--gpus 1] [--steps 4] [--warmup 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
TUNE_CACHE = os.path.join(ROOT, "paper_2504_17881_amd", "tuning", "gfx950.json")
METRIC = "amplitude-updates/s and %HBM peak at n=32, FP32-fused vs FP64-plain"


def kernel_symbol(ps: dict, dtype_name: str) -> str:
    if ps["kind"] == 1:
        return f"k_span<{dtype_name},{ps['m']}>"
    if ps["kind"] == 2:
        return f"k_tile<{dtype_name},{ps['B']},{ps['m']}>"
    if ps["kind"] == 3:
        return f"k_permute<{dtype_name}>"
    return f"k_plain<{dtype_name}>"


def kernel_sources_digest() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "device.h", "internal.h", "rot_jump_f32m4.inc",
              "rot_loop_f32m4.inc", "rot_jump_f64m4.inc", "rot_loop_f64m4.inc"):
        with open(os.path.join(ROOT, "paper_2504_17881_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_value(fname: str, kernel: str, key: str):
    """A `key = value` line of a committed rocprofv3 counter summary under
    profiles/, if the summary was taken on the current kernel sources and
    for `kernel`; else None."""
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        line = line.lstrip("# ").rstrip()
        if " = " in line:
            k, v = line.split(" = ", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sources") != kernel_sources_digest():
        return None
    if vals.get("kernel") != kernel:
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def limiter(hbm_frac: float, valu_busy):
    """The unit that the counters show closest to saturation for the dominant
    kernel: "valu" when its vector ALU busy fraction (shader counters) is
    above its HBM fraction of peak, else "hbm"; "hbm" without counters."""
    if valu_busy is not None and valu_busy > hbm_frac:
        return "valu"
    return "hbm"


def read_traffic(kernel: str):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) from the
    committed counter summary, if taken on the current kernel sources."""
    return _profile_value("traffic_trotter1_n32_c64.txt", kernel, "hbm_bytes_per_launch")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(x, z, phi, n: int, k0: int, budget_s: float, max_rot: int):
    """Applies rotation 0 untimed (it also first-touches the state and the
    oracle's scratch array), then rotations 1, 2, ... one by one until the
    budget is spent; returns (timed rotations, seconds, threads)."""
    import numpy as np
    sys.path.insert(0, ROOT)
    from oracle import statevector as sv
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[k0] = 1.0
    work = np.empty_like(psi)
    sv.c_apply_rotations(psi, x[0:1], z[0:1], phi[0:1], out=psi, work=work)
    done = 0
    t0 = time.perf_counter()
    while done < max_rot:
        r = done + 1
        sv.c_apply_rotations(psi, x[r:r + 1], z[r:r + 1], phi[r:r + 1], out=psi, work=work)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    return done, time.perf_counter() - t0, sv.c_threads()


def _trotter1_n28_rotations():
    """The n = 28 Trotter workload's schedule (given term order), re-expanded
    by the oracle's schedule builder."""
    sys.path.insert(0, ROOT)
    import synth
    from oracle import schedules as osch
    w = synth.WORKLOADS["trotter1_n28"]
    x, z, h = synth.jw_hamiltonian(w["n"], w["L"], w["ham_seed"])
    rx, rz, rp = osch.trotter(x, z, h, 1, w["t"], w["steps"], suffix=False)
    return w["n"], rx, rz, rp, synth.basis_index(w["n"])


def full_small_runs():
    """The oracle on two whole small workloads, all cores: the 14-qubit
    random-rotation case (1000 rotations from a Gaussian state) and the
    n = 20 check of the n = 32 Trotter workload (same H recipe with its own
    seed, 4 steps of 5000 rotations)."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import synth
    from oracle import schedules as osch
    from oracle import statevector as sv
    out = {}
    w = synth.WORKLOADS["random_n14"]
    x, z, phi = synth.random_pauli_rotations(w["n"], w["M"], w["rot_seed"])
    psi = synth.gaussian_state(w["n"], w["state_seed"])
    t0 = time.perf_counter()
    sv.c_apply_rotations(psi, x, z, phi, out=psi)
    dt = time.perf_counter() - t0
    out["random_n14"] = {"rotations": int(w["M"]), "seconds": dt,
                         "value": w["M"] * float(1 << w["n"]) / dt, "cores": sv.c_threads()}
    w = synth.WORKLOADS["trotter1_n32"]
    n = w["check_n"]
    x, z, h = synth.jw_hamiltonian(n, w["L"], w["check_seed"])
    rx, rz, rp = osch.trotter(x, z, h, 1, w["t"], w["steps"], suffix=True)
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[synth.basis_index(n)] = 1.0
    t0 = time.perf_counter()
    sv.c_apply_rotations(psi, rx, rz, rp, out=psi)
    dt = time.perf_counter() - t0
    out["trotter1_n20_check"] = {"rotations": len(rx), "seconds": dt,
                                 "value": len(rx) * float(1 << n) / dt,
                                 "cores": sv.c_threads()}
    return out


def one_core_worker(budget_s: float) -> int:
    """Child process (OMP_NUM_THREADS=1): the oracle on one core, first
    rotations of the n = 28 Trotter workload; prints one JSON line."""
    n, rx, rz, rp, k0 = _trotter1_n28_rotations()
    done, dt, thr = _oracle_rate(rx, rz, rp, n, k0, budget_s, 100)
    print(json.dumps({"rotations": done, "seconds": dt, "threads": thr, "n": n}))
    return 0


def cpu_baseline(x, z, phi, n: int, k0: int, budget_s: float, max_rot: int):
    """The oracle as it stands: all cores on the first rotations of the
    benchmark schedule; one core (child process) and all cores on the n = 28
    Trotter workload's first rotations (at most 100); all cores on two whole
    small workloads (full_small_runs)."""
    import subprocess
    done, dt, thr = _oracle_rate(x, z, phi, n, k0, budget_s, max_rot)
    out = {
        "value": done * float(1 << n) / dt,
        "unit": "amplitude-updates/s",
        "cores": thr,
        "kind": "oracle",
        "sample": (f"rotations 1..{done} of the same n={n} schedule from the same basis "
                   f"state (rotation 0 untimed), FP64 C oracle (scatter form, OpenMP), "
                   f"{dt:.1f} s"),
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
    }
    n28, rx, rz, rp, b28 = _trotter1_n28_rotations()
    d2, t2, thr2 = _oracle_rate(rx, rz, rp, n28, b28, budget_s, 100)
    out["n28_rate"] = {"value": d2 * float(1 << n28) / t2, "cores": thr2, "rotations": d2,
                       "seconds": t2, "sample": "rotations 1.. of the n=28 Trotter workload (rotation 0 untimed)"}
    out["full_runs"] = full_small_runs()
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--one-core-worker",
                        "--cpu-budget", str(budget_s / 2)], env=env, capture_output=True,
                       text=True, timeout=600)
    if r.returncode == 0 and r.stdout.strip():
        one = json.loads(r.stdout.strip().splitlines()[-1])
        out["one_core"] = {"value": one["rotations"] * float(1 << one["n"]) / one["seconds"],
                           "cores": one["threads"], "rotations": one["rotations"],
                           "seconds": one["seconds"],
                           "sample": "rotations 1.. of the n=28 Trotter workload (rotation 0 untimed)"}
    return out


def fusion_sweep(ns, reps: int) -> int:
    """Fusion-depth curve: groups of L = 1, 10, 100 rotations that share one
    high X part (random low X and Z parts, angles U[-pi, pi]), applied as one
    sweep per rotation (plain) and as fused passes, at several n and both
    precisions.  One JSON line per (dtype, n, L, kernel) with the time per
    rotation and the HBM traffic of the passes against the 8 TB/s peak."""
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    from paper_2504_17881_amd import prx as P
    dev = torch.device("cuda:0")
    low = 8  # the shared high X part starts above every tile's low qubits
    for dt, name, s in ((P.PRX_C64, "c64", 8), (P.PRX_C128, "c128", 16)):
        for n in ns:
            psi = torch.zeros(1 << n, dtype=torch.complex64 if s == 8 else torch.complex128,
                              device=dev)
            psi[0] = 1.0
            for L in (1, 10, 100):
                rng = np.random.default_rng(1000 * n + L)
                xh = int(rng.integers(1, 1 << (n - low)))
                x = ((np.uint64(xh) << np.uint64(low)) |
                     rng.integers(0, 1 << low, size=L).astype(np.uint64)).astype(np.uint64)
                z = rng.integers(0, 1 << n, size=L, dtype=np.uint64)
                phi = rng.uniform(-np.pi, np.pi, size=L)
                sched = P.prx_sched_from_rotations(n, x, z, phi)
                for kern, kname in ((P.PRX_PLAIN, "plain"), (P.PRX_FUSED, "fused")):
                    pl = P.prx_plan_create(sched, n, dt, 0, L, kern)
                    info = P.prx_plan_get_info(pl)
                    ws = torch.empty(max(info["workspace_bytes"], 256), dtype=torch.uint8,
                                     device=dev)
                    P.prx_plan_upload(pl, ws)
                    P.prx_plan_execute_timed(pl, psi, ws)  # warm-up
                    tot = 0.0
                    for _ in range(reps):
                        pm, rm = P.prx_plan_execute_timed(pl, psi, ws)
                        tot += float(pm.sum()) + float(rm.sum())
                    ms = tot / reps
                    nbytes = info["passes"] * 2.0 * (1 << n) * s
                    print(json.dumps({"dtype": name, "n": n, "L": L, "kernel": kname,
                                      "passes": info["passes"], "ms": ms,
                                      "ms_per_rotation": ms / L,
                                      "updates_per_s": L * float(1 << n) / (ms * 1e-3),
                                      "hbm_frac": nbytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)}),
                          flush=True)
                    P.prx_plan_destroy(pl)
                    del ws
                P.prx_sched_destroy(sched)
            del psi
            torch.cuda.empty_cache()
    return 0


def relabel_compare(reps: int) -> int:
    """Qubit relabelling against none, on random-order sequences (one JSON line
    each): a qDRIFT sample of the batching workload's n = 24 Hamiltonian
    (2000 draws, complex64, 14-qubit tile-sets) and the random part of one
    step of the large-state workload (n = 34, 1000 draws, complex64, 12- and
    14-qubit tile-sets): passes, relabelling passes and the time per
    application (HIP events around every pass, best of `reps`)."""
    import torch
    sys.path.insert(0, ROOT)
    import synth
    from paper_2504_17881_amd import prx as P
    dev = torch.device("cuda:0")
    cases = []
    x, z, h = synth.jw_hamiltonian(24, 500, 1024)
    H24 = P.prx_ham_create(24, x, z, h)
    cases.append(("qdrift_n24", 24, P.prx_sched_qdrift(H24, 1.0, 2000, 3), 0, 2000, 14, 10))
    w = synth.WORKLOADS["partial_n34"]
    x, z, h = synth.jw_hamiltonian(34, w["L"], w["ham_seed"])
    H34 = P.prx_ham_create(34, x, z, h)
    s34 = P.prx_sched_partial(H34, w["L_det"], w["t"], w["steps"], w["r"], 0,
                              P.PRX_REORDER_SUFFIX)
    r0 = w["L_det"]  # step 1: D forward, then the random draws
    for B, G in ((12, 8), (14, 10)):
        cases.append((f"partial_n34_random_step1_B{B}", 34, s34, r0, r0 + w["r"], B, G))
    for name, n, sch, b, e, B, G in cases:
        psi = torch.zeros(1 << n, dtype=torch.complex64, device=dev)
        psi[synth.basis_index(n)] = 1.0
        for rl in (0, 1):
            pl = P.prx_plan_create(sch, n, P.PRX_C64, b, e, P.PRX_FUSED,
                                   dict(tile_qubits=B, max_virtual=G, relabel=rl))
            info = P.prx_plan_get_info(pl)
            ws = torch.empty(max(info["workspace_bytes"], 256), dtype=torch.uint8, device=dev)
            P.prx_plan_upload(pl, ws)
            P.prx_plan_execute_timed(pl, psi, ws)
            best = None
            for _ in range(max(1, reps)):
                pm, rm = P.prx_plan_execute_timed(pl, psi, ws)
                ms = float(pm.sum() + rm.sum())
                best = ms if best is None else min(best, ms)
            print(json.dumps({"case": name, "n": n, "rotations": e - b, "tile_qubits": B,
                              "relabel": rl, "passes": info["passes"],
                              "relabel_passes": info["relabel_passes"], "ms": best}),
                  flush=True)
            P.prx_plan_destroy(pl)
            del ws
        del psi
        torch.cuda.empty_cache()
    P.prx_sched_destroy(cases[0][2])
    P.prx_sched_destroy(s34)
    P.prx_ham_destroy(H24)
    P.prx_ham_destroy(H34)
    return 0


def batch_workload(steps: int, warmup: int) -> int:
    """The batching workload: 256 qDRIFT samples with n uniform on 16..24
    (per-size JW Hamiltonian, L = 500, N = 2000 draws, t = 1), complex64,
    basis initial states, all samples in one captured graph.  A step is one
    graph launch (every sample's full sequence and the overlap read-out),
    timed with HIP events on its stream; the states are reset between
    steps, outside the timed region.  One JSON line: samples/s, and the
    algorithmic HBM traffic (every pass reads and writes its sample once)
    against the 8 TB/s peak."""
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    import synth
    from paper_2504_17881_amd import prx as P
    dev = torch.device("cuda:0")
    w = synth.WORKLOADS["qdrift_batch"]
    ns = synth.batch_qubit_counts(w["S"], w["n_lo"], w["n_hi"], w["n_seed"])
    hams, scheds = {}, []
    for i, n in enumerate(ns):
        if n not in hams:
            x, z, h = synth.jw_hamiltonian(n, w["L"], 1000 + n)
            hams[n] = P.prx_ham_create(n, x, z, h)
        scheds.append(P.prx_sched_qdrift(hams[n], w["t"], w["N"], i))
    basis = [synth.basis_index(n) for n in ns]
    psis = [torch.zeros(1 << n, dtype=torch.complex64, device=dev) for n in ns]
    b = P.prx_batch_create(ns, scheds, P.PRX_C64, basis)
    info = P.prx_batch_get_info(b)
    ws = torch.empty(P.prx_batch_workspace_bytes(b), dtype=torch.uint8, device=dev)
    ovd = torch.zeros(2 * len(ns), dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream()
    P.prx_batch_upload(b, psis, ws, stream=stream)
    g = P.prx_batch_graph(b, ws, ovd, stream)
    print(f"[bench] qdrift batch: S={len(ns)} rounds={info['rounds']} passes={info['passes']} "
          f"tile samples={info['tile_samples']}", file=sys.stderr, flush=True)
    total_ms = 0.0
    for it in range(warmup + steps):
        for t, k in zip(psis, basis):
            t.zero_()
            t[k] = 1.0
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.prx_graph_launch(g, stream)
        e1.record(stream)
        stream.synchronize()
        ms = e0.elapsed_time(e1)
        if it >= warmup:
            total_ms += ms
        print(f"[bench] batch step {it} ({'warm-up' if it < warmup else 'timed'}): {ms:.1f} ms",
              file=sys.stderr, flush=True)
    ov = ovd.cpu().numpy()
    ms = total_ms / max(1, steps)
    gbs = 2.0 * info["amp_sweeps"] * 8 / (ms * 1e-3) / 1e9
    print(json.dumps({
        "metric": "qDRIFT batch throughput (256 samples, n 16-24, N = 2000, complex64)",
        "value": len(ns) / (ms * 1e-3), "unit": "samples/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "qdrift_batch", "S": len(ns), "n_lo": w["n_lo"],
                   "n_hi": w["n_hi"], "L": w["L"], "N": w["N"], "t": w["t"],
                   "tile_samples": info["tile_samples"], "rounds": info["rounds"],
                   "passes": info["passes"], "amp_sweeps": info["amp_sweeps"]},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "kernel": "whole graph (all rounds)"},
        "mean_overlap": [float(np.mean(ov[0::2])), float(np.mean(ov[1::2]))],
    }), flush=True)
    P.prx_graph_destroy(g)
    P.prx_batch_destroy(b)
    for s in scheds:
        P.prx_sched_destroy(s)
    for H in hams.values():
        P.prx_ham_destroy(H)
    return 0


def _diff_norm(a, b, chunk=1 << 26) -> float:
    """||a - b||_2 in FP64, chunk by chunk (no full-size temporaries)."""
    import torch
    acc = 0.0
    for s0 in range(0, a.numel(), chunk):
        d = a[s0:s0 + chunk].to(torch.complex128) - b[s0:s0 + chunk].to(torch.complex128)
        acc += float(torch.sum(d.real * d.real + d.imag * d.imag))
    return acc ** 0.5


def _dominant(per_kernel: dict):
    name, (cnt, ms) = max(per_kernel.items(), key=lambda kv: kv[1][1])
    return name, cnt, ms / cnt


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--plain-rotations", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--fused-only", action="store_true",
                    help="skip the FP64-plain comparator and the precision leg (profiling runs)")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the complex64-against-complex128 whole-run leg")
    ap.add_argument("--one-core-worker", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="autotune cache (JSON) loaded before planning; plans use PRX_AUTO")
    ap.add_argument("--autotune-save", default=None,
                    help="run the autotuner on the first --tune-rotations rotations first and "
                         "save its cache to this path")
    ap.add_argument("--tune-rotations", type=int, default=5000,
                    help="rotations of the schedule timed per autotune setting (default: one Trotter step)")
    ap.add_argument("--tune-dtype", choices=("c64", "c128"), default="c64",
                    help="state precision the autotuner times (the saved cache keeps the other "
                         "entries of --tune-cache)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="GIB",
                    help="first run torch copies of GIB GiB (3 launches): the known-size "
                         "reference that scales hardware byte counters")
    ap.add_argument("--fusion-sweep", action="store_true",
                    help="instead of the benchmark, print the fusion-depth curve (plain against "
                         "fused for groups of 1, 10, 100 rotations sharing a high X part)")
    ap.add_argument("--sweep-n", default="16,20,24,28,32")
    ap.add_argument("--batch-workload", action="store_true",
                    help="instead of the benchmark, time the qDRIFT batching workload "
                         "(256 samples in one graph)")
    ap.add_argument("--relabel-compare", action="store_true",
                    help="instead of the benchmark, compare plans with and without qubit "
                         "relabelling on random-order sequences")
    args = ap.parse_args()
    if args.one_core_worker:
        return one_core_worker(args.cpu_budget)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the hot path is a "
              "single-device kernel and this build has no multi-GPU path.", file=sys.stderr)
        return 2
    if args.fusion_sweep:
        return fusion_sweep([int(v) for v in args.sweep_n.split(",")], max(1, args.steps))
    if args.batch_workload:
        return batch_workload(max(1, args.steps), max(0, args.warmup))
    if args.relabel_compare:
        return relabel_compare(max(1, args.steps))

    import numpy as np
    sys.path.insert(0, ROOT)
    import synth

    w = synth.WORKLOADS["trotter1_n32"]
    n = args.n
    L, t, S = w["L"], w["t"], w["steps"]
    x, z, h = synth.jw_hamiltonian(n, L, w["ham_seed"])
    k0 = synth.basis_index(n)

    # ---------------- CPU baseline first, before anything touches the GPU
    # (its one-core leg runs in a child process)
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import schedules as osch
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        ox, oz, op = osch.trotter(x, z, h, 1, t, S, suffix=True)
        cpu = cpu_baseline(ox, oz, op, n, k0, args.cpu_budget, 4)
        del ox, oz, op

    import torch
    from paper_2504_17881_amd import prx as P

    H = P.prx_ham_create(n, x, z, h)
    sched = P.prx_sched_trotter(H, 1, t, S, P.PRX_REORDER_SUFFIX)
    _, sx, sz, sphi = P.prx_sched_view(sched)
    dev = torch.device("cuda:0")
    print(f"[bench] n={n} L={L} rotations={len(sx)}", file=sys.stderr, flush=True)

    if args.copy_calibration:
        nbytes = args.copy_calibration << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 3 copies of {nbytes} B (read {nbytes} B, "
              f"write {nbytes} B each)", file=sys.stderr, flush=True)
        del src, dst
        torch.cuda.empty_cache()

    # ---------------- planner settings: tuned cache (or a fresh tuning run)
    if args.tune_cache and os.path.exists(args.tune_cache):
        P.prx_autotune_load(args.tune_cache)
    if args.autotune_save:
        print(f"[bench] autotuning {args.tune_dtype}", file=sys.stderr, flush=True)
        R = min(args.tune_rotations, len(sx))
        sub = P.prx_sched_from_rotations(n, sx[:R], sz[:R], sphi[:R])
        tdt = P.PRX_C64 if args.tune_dtype == "c64" else P.PRX_C128
        scratch = torch.zeros(1 << n, dtype=torch.complex64 if tdt == P.PRX_C64
                              else torch.complex128, device=dev)
        scratch[k0] = 1.0
        tws = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        def _trial(o, ms):
            print(f"[bench] tune {({k: v for k, v in o.items() if v})} {ms:.1f} ms",
                  file=sys.stderr, flush=True)
        best, trials = P.prx_autotune(scratch, n, tdt, sub, tws, progress=_trial)
        os.makedirs(os.path.dirname(os.path.abspath(args.autotune_save)), exist_ok=True)
        P.prx_autotune_save(args.autotune_save)
        print(f"[bench] autotune: {trials} trials, best {best}", file=sys.stderr, flush=True)
        P.prx_sched_destroy(sub)
        del scratch, tws
        torch.cuda.empty_cache()
    tuned = P.prx_autotune_lookup(n, P.PRX_C64)
    kernel = P.PRX_AUTO if tuned else P.PRX_FUSED

    # ---------------- fused complex64: one plan per Trotter step (identical steps)
    plan = P.prx_plan_create(sched, n, P.PRX_C64, 0, L, kernel)
    info = P.prx_plan_get_info(plan)
    passes = [P.prx_plan_pass(plan, i) for i in range(info["passes"])]
    names = [kernel_symbol(p, "float") for p in passes]
    ws = torch.empty(info["workspace_bytes"], dtype=torch.uint8, device=dev)
    P.prx_plan_upload(plan, ws)
    psi = torch.zeros(1 << n, dtype=torch.complex64, device=dev)
    psi[k0] = 1.0
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        P.prx_plan_execute_timed(plan, psi, ws)
        P.prx_amplitude(psi, n, P.PRX_C64, k0)
    # the timed steps start from the workload's initial state
    psi.zero_()
    psi[k0] = 1.0
    torch.cuda.synchronize()
    print(f"[bench] fused c64: {info['passes']} passes/step, mean fuse "
          f"{info['mean_fuse']:.2f}", file=sys.stderr, flush=True)

    per_kernel = {}
    renorm_total = 0.0
    ovs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pm, rm = P.prx_plan_execute_timed(plan, psi, ws)
        ovs.append(P.prx_amplitude(psi, n, P.PRX_C64, k0))  # <k0|psi>
        for nm, ms in zip(names, pm):
            a = per_kernel.setdefault(nm, [0, 0.0])
            a[0] += 1
            a[1] += float(ms)
        renorm_total += float(rm.sum())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    updates = args.steps * L * float(1 << n)
    value = updates / wall
    bytes_per_pass = 2.0 * float(1 << n) * 8
    dom_name, dom_cnt, dom_avg_ms = _dominant(per_kernel)
    achieved = bytes_per_pass / (dom_avg_ms * 1e-3) / 1e9
    traffic = read_traffic(dom_name)
    valu_busy = _profile_value("sq_counters_trotter1_n32_c64.md", dom_name, "valu_busy")
    all_pass_bw = args.steps * info["passes"] * bytes_per_pass / wall / 1e9
    del psi
    torch.cuda.empty_cache()
    print(f"[bench] timed: {wall / args.steps * 1e3:.1f} ms per step, {dom_name} "
          f"{dom_avg_ms:.2f} ms per launch", file=sys.stderr, flush=True)

    # ---------------- precision leg (outside the timed region): the whole run
    # in complex64 fused against complex128 fused, both resident
    precision = None
    if not (args.fused_only or args.no_precision):
        print("[bench] precision leg: complex64 against complex128 over the whole run",
              file=sys.stderr, flush=True)
        tuned128 = P.prx_autotune_lookup(n, P.PRX_C128)
        plan128 = P.prx_plan_create(sched, n, P.PRX_C128, 0, L,
                                    P.PRX_AUTO if tuned128 else P.PRX_FUSED)
        info128 = P.prx_plan_get_info(plan128)
        names128 = [kernel_symbol(P.prx_plan_pass(plan128, i), "double")
                    for i in range(info128["passes"])]
        ws128 = torch.empty(info128["workspace_bytes"], dtype=torch.uint8, device=dev)
        P.prx_plan_upload(plan128, ws128)
        a = torch.zeros(1 << n, dtype=torch.complex64, device=dev)
        b = torch.zeros(1 << n, dtype=torch.complex128, device=dev)
        a[k0] = 1.0
        b[k0] = 1.0
        torch.cuda.synchronize()
        rows, k128, wall128 = [], {}, 0.0
        for step in range(1, S + 1):
            P.prx_plan_execute_timed(plan, a, ws)
            tb0 = time.perf_counter()
            pm, _ = P.prx_plan_execute_timed(plan128, b, ws128)
            wall128 += time.perf_counter() - tb0
            for nm, ms in zip(names128, pm):
                e = k128.setdefault(nm, [0, 0.0])
                e[0] += 1
                e[1] += float(ms)
            if step * L == 10000 or step == S:
                oa = P.prx_amplitude(a, n, P.PRX_C64, k0)
                ob = P.prx_amplitude(b, n, P.PRX_C128, k0)
                rows.append({"rotations": step * L, "err_l2": _diff_norm(a, b),
                             "d_overlap": abs(oa - ob), "overlap_c128": [ob.real, ob.imag],
                             "overlap_c64": [oa.real, oa.imag]})
                print(f"[bench] precision at {step * L} rotations: err_l2 "
                      f"{rows[-1]['err_l2']:.3e} |d overlap| {rows[-1]['d_overlap']:.3e}",
                      file=sys.stderr, flush=True)
        d128, c128, avg128 = _dominant(k128)
        bpp128 = 2.0 * float(1 << n) * 16
        ach128 = bpp128 / (avg128 * 1e-3) / 1e9
        precision = {
            "reference": "complex128 fused (tuned) over the same schedule from the same state",
            "at": rows,
            "err_l2": rows[-1]["err_l2"], "d_overlap": rows[-1]["d_overlap"],
            "fp64_fused": {
                "value": S * L * float(1 << n) / wall128, "unit": "amplitude-updates/s",
                "passes_per_step": info128["passes"],
                "planner": ({k: v for k, v in tuned128.items() if v} if tuned128
                            else "defaults"),
                "roofline": {"bound": "hbm", "achieved": ach128, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": ach128 / HBM_PEAK_GBS, "kernel": d128,
                             "launches": c128, "avg_launch_ms": avg128,
                             "bytes_per_launch": bpp128},
            },
        }
        P.prx_plan_destroy(plan128)
        del a, b, ws128
        torch.cuda.empty_cache()
    P.prx_plan_destroy(plan)
    del ws
    torch.cuda.empty_cache()

    # ---------------- FP64 plain comparator (complex128, one sweep per rotation)
    fp64 = None
    if not args.fused_only:
        R = min(args.plain_rotations, len(sx))
        pplan = P.prx_plan_create(sched, n, P.PRX_C128, 0, R, P.PRX_PLAIN)
        pinfo = P.prx_plan_get_info(pplan)
        pws = torch.empty(pinfo["workspace_bytes"], dtype=torch.uint8, device=dev)
        P.prx_plan_upload(pplan, pws)
        psi2 = torch.zeros(1 << n, dtype=torch.complex128, device=dev)
        psi2[k0] = 1.0
        warm = P.prx_plan_create(sched, n, P.PRX_C128, 0, 4, P.PRX_PLAIN)
        wws = torch.empty(P.prx_plan_get_info(warm)["workspace_bytes"], dtype=torch.uint8,
                          device=dev)
        P.prx_plan_upload(warm, wws)
        P.prx_plan_execute(warm, psi2, wws)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        pm, _ = P.prx_plan_execute_timed(pplan, psi2, pws)
        torch.cuda.synchronize()
        pwall = time.perf_counter() - tp0
        p_updates = R * float(1 << n)
        avg_ms = float(pm.mean())
        fp64 = {
            "value": p_updates / pwall,
            "unit": "amplitude-updates/s",
            "rotations": R,
            "kernel": "k_plain_pair<double,4> / k_plain_diag<double,4>",
            "avg_launch_ms": avg_ms,
            "hbm_frac": (2.0 * float(1 << n) * 16 / (avg_ms * 1e-3) / 1e9) / HBM_PEAK_GBS,
            "fused_c64_over_plain_c128": value / (p_updates / pwall),
        }
        P.prx_plan_destroy(pplan)
        P.prx_plan_destroy(warm)
        del psi2, pws, wws
        torch.cuda.empty_cache()

    run_steps = min(S, args.steps)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "amplitude-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"trotter1_n{n}: synthetic JW-shaped H, n={n}, L={L}, first-order "
                         f"Trotter t={t}, {S} steps ({S * L} rotations), lexicographic (SUFFIX) "
                         "term order, from the basis state with the low 16 bits set; complex64 "
                         "fused with FP64 renormalisation.  One bench step = one Trotter step "
                         f"({L} rotations; every step is the same product) + the basis "
                         f"overlap; the timed loop applies {args.steps} consecutive steps to "
                         f"one state (steps 1-{S} are the workload's run, later steps "
                         "continue it)"),
            "n": n, "L": L, "rotations_per_step": L,
            "passes_per_step": info["passes"], "mean_fuse": info["mean_fuse"],
            "span_passes": info["span_passes"], "tile_passes": info["tile_passes"],
            "plain_passes": info["plain_passes"],
            "planner": ({k: v for k, v in tuned.items() if v} if tuned else "defaults"),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "valu_busy": valu_busy,
            "limiter": limiter(achieved / HBM_PEAK_GBS, valu_busy),
            "kernel": dom_name,
            "launches": dom_cnt,
            "avg_launch_ms": dom_avg_ms,
            "bytes_per_launch": bytes_per_pass,
            "all_passes_GBps": all_pass_bw,
        },
        "kernels": {k: {"launches": c, "total_ms": ms, "avg_ms": ms / c}
                    for k, (c, ms) in sorted(per_kernel.items())},
        "renorm_ms_total": renorm_total,
        "overlap_run_end": ([ovs[run_steps - 1].real, ovs[run_steps - 1].imag]
                            if args.steps >= S else None),
        "overlap_last_step": [ovs[-1].real, ovs[-1].imag] if ovs else None,
        "err_l2": precision["err_l2"] if precision else None,
        "d_overlap": precision["d_overlap"] if precision else None,
        "precision": precision,
        "fp64_plain": fp64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
