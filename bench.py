#!/usr/bin/env python3
"""Benchmark: amplitude updates/s and HBM roofline at n=32, FP32 fused vs FP64 plain.

Workload (precision workload): synthetic Jordan-Wigner-shaped Hamiltonian,
n = 32, L = 5000 terms (seed 0), lexicographically ordered terms,
first-order Trotter with t = 0.5 and 4 steps (2*10^4 rotations), initial
basis state with the low 16 bits set.  One bench step is one Trotter step
(5000 rotations) applied by the fused complex64 path with FP64
renormalisation, followed by the overlap with the initial basis state.

Reported:
  value        amplitude updates per second of the timed steps
               (updates = rotations * 2^n; inputs resident in HBM);
  roofline     the dominant kernel (largest share of the timed steps'
               kernel time): algorithmic bytes per launch (2 * 2^n * 8 B,
               one read and one write of the state) over its average
               launch duration from HIP events recorded around every pass;
  fp64_plain   the complex128 single-rotation sweep on the same schedule
               (first `--plain-rotations` rotations), for the 2x comparison;
  cpu_baseline the FP64 CPU oracle on the first rotations of the same
               schedule and state, on this host's cores.

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
    return f"k_plain<{dtype_name}>"


def kernel_sources_digest() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "device.h", "internal.h", "rot_jump_f32m4.inc"):
        with open(os.path.join(ROOT, "paper_2504_17881_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_trotter1_n32_c64.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_sources") != kernel_sources_digest():
        return None
    if vals.get("kernel") != kernel:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(x, z, phi, n: int, k0: int, budget_s: float, max_rot: int):
    """The oracle as it stands, on the first rotations of the schedule."""
    import numpy as np
    sys.path.insert(0, ROOT)
    from oracle import statevector as sv
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[k0] = 1.0
    work = np.empty_like(psi)
    done = 0
    t0 = time.perf_counter()
    while done < max_rot:
        sv.c_apply_rotations(psi, x[done:done + 1], z[done:done + 1], phi[done:done + 1],
                             out=psi, work=work)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {
        "value": done * float(1 << n) / dt,
        "unit": "amplitude-updates/s",
        "cores": sv.c_threads(),
        "kind": "oracle",
        "sample": (f"first {done} rotation(s) of the same n={n} schedule from the same basis "
                   f"state, FP64 C oracle (scatter form, OpenMP), {dt:.1f} s"),
    }


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
                    help="skip the FP64-plain comparator (profiling runs)")
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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the hot path is a "
              "single-device kernel and this build has no multi-GPU path.", file=sys.stderr)
        return 2
    if args.fusion_sweep:
        return fusion_sweep([int(v) for v in args.sweep_n.split(",")], max(1, args.steps))
    if args.batch_workload:
        return batch_workload(max(1, args.steps), max(0, args.warmup))

    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    import synth
    from paper_2504_17881_amd import prx as P

    w = synth.WORKLOADS["trotter1_n32"]
    n = args.n
    L, t, S = w["L"], w["t"], w["steps"]
    x, z, h = synth.jw_hamiltonian(n, L, w["ham_seed"])
    H = P.prx_ham_create(n, x, z, h)
    sched = P.prx_sched_trotter(H, 1, t, S, P.PRX_REORDER_SUFFIX)
    _, sx, sz, sphi = P.prx_sched_view(sched)
    k0 = synth.basis_index(n)
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
    tuned = None
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
    bra = k0
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        P.prx_plan_execute_timed(plan, psi, ws)
        P.prx_amplitude(psi, n, P.PRX_C64, bra)
    torch.cuda.synchronize()
    print(f"[bench] fused c64: {info['passes']} passes/step, mean fuse "
          f"{info['mean_fuse']:.2f}", file=sys.stderr, flush=True)

    per_kernel = {}
    renorm_total = 0.0
    ov = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pm, rm = P.prx_plan_execute_timed(plan, psi, ws)
        ov = P.prx_amplitude(psi, n, P.PRX_C64, bra)  # <k0|psi>
        for nm, ms in zip(names, pm):
            a = per_kernel.setdefault(nm, [0, 0.0])
            a[0] += 1
            a[1] += float(ms)
        renorm_total += float(rm.sum())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    updates = args.steps * L * float(1 << n)
    value = updates / wall
    state_bytes = float(1 << n) * 8
    bytes_per_pass = 2.0 * state_bytes
    dom = max(per_kernel.items(), key=lambda kv: kv[1][1])
    dom_name, (dom_cnt, dom_ms) = dom
    dom_avg_ms = dom_ms / dom_cnt
    achieved = bytes_per_pass / (dom_avg_ms * 1e-3) / 1e9
    traffic = read_traffic(dom_name)
    all_pass_bw = args.steps * info["passes"] * bytes_per_pass / wall / 1e9
    P.prx_plan_destroy(plan)
    del psi, ws
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

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(sx, sz, sphi, n, k0, args.cpu_budget, 4)

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
                         f"Trotter t={t}, {S} steps in the run, lexicographic (SUFFIX) term "
                         "order, complex64 fused with FP64 renormalisation; one step = one "
                         "Trotter step (5000 rotations) + basis overlap"),
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
            "kernel": dom_name,
            "launches": dom_cnt,
            "avg_launch_ms": dom_avg_ms,
            "bytes_per_launch": bytes_per_pass,
            "all_passes_GBps": all_pass_bw,
        },
        "kernels": {k: {"launches": c, "total_ms": ms, "avg_ms": ms / c}
                    for k, (c, ms) in sorted(per_kernel.items())},
        "renorm_ms_total": renorm_total,
        "overlap_final": [ov.real, ov.imag] if ov is not None else None,
        "fp64_plain": fp64,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
