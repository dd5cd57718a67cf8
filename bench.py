"""Benchmark: SSA events/s on one MI355X for the Schloegl ensemble
(100,000 trajectories, T_end = 10, 101 snapshots), mixed FP16 with
stochastic rounding (the reported value) against the FP64 direct method.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one complete ensemble run (every trajectory from t = 0 to T_end:
RNG draws, propensities, sums, waiting times, snapshot stores, selection and
integer updates) through the C ABI. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_VALU_SLOTS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock: full-rate VALU lane slots/s


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--mode", default="MIX_F16_SR")
    p.add_argument("--ref-mode", default="FP64")
    p.add_argument("--n-traj", type=int, default=100_000)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=4000, help="trajectories the oracle runs for cpu_baseline")
    p.add_argument("--verbose", action="store_true")
    return p.parse_args()


def timed_runs(ssa, items, W, mode, steps, warmup, log):
    import torch
    for _ in range(warmup):
        r = ssa.ssa_ensemble_run(items, W.t_end, W.snap_t, W.seed, mode, max_events=W.max_events)
        r.wait()
        del r
    torch.cuda.synchronize()
    runs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        runs.append(ssa.ssa_ensemble_run(items, W.t_end, W.snap_t, W.seed, mode, max_events=W.max_events))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    infos = [r.info() for r in runs]
    events = sum(i["total_events"] for i in infos)
    kern_ms = [i["kernel_ms"] for i in infos]
    log(f"[bench] {mode}: {steps} steps, {events} events, wall {wall:.3f}s, kernel ms {kern_ms}")
    last = runs[-1]
    x_end = last.snapshots(0)[-1, 0].copy()
    st = last.stats(0)
    return {"wall_s": wall, "events": events, "events_per_step": events / steps,
            "kernel_ms_avg": float(np.mean(kern_ms)), "info": infos[-1], "x_end": x_end,
            "status_counts": np.bincount(st["status"], minlength=4).tolist()}


def cpu_baseline(W, mode, n_sample, log):
    import oracle
    threads = min(16, os.cpu_count() or 1)
    it = W.items[0]
    idx = np.arange(n_sample, dtype=np.int64)
    t0 = time.perf_counter()
    r = oracle.simulate(it.model, mode, it.x0, W.t_end, W.snap_t, W.seed, indices=idx,
                        max_events=W.max_events, threads=threads)
    dt = time.perf_counter() - t0
    ev = int(r["n_events"].sum())
    log(f"[bench] cpu oracle {mode}: {n_sample} trajectories, {ev} events in {dt:.2f}s on {threads} threads")
    return {"value": ev / dt, "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": f"trajectories 0..{n_sample - 1} of the same Schloegl ensemble, {mode}, full horizon"}


def main():
    args = parse()
    log = (lambda m: print(m, file=sys.stderr, flush=True))
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the path has no multi-GPU part); got --gpus {args.gpus}",
              file=sys.stderr)
        return 2
    import torch
    from paper_2605_00479_amd import ssa, stats, workloads as wl
    from paper_2605_00479_amd.csrc import valu_count
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    ssa.lib()
    W = wl.config_schlogl(args.n_traj)
    items = ssa.items_from_workload(W)
    log(f"[bench] workload schlogl: {W.n_traj} trajectories, T_end {W.t_end}, {len(W.snap_t)} snapshots")

    main_res = timed_runs(ssa, items, W, args.mode, args.steps, args.warmup, log)
    ref_res = timed_runs(ssa, items, W, args.ref_mode, args.steps, args.warmup, log)

    # fidelity of the end-time ensemble (species X at T_end) against FP64:
    # independent seeds for the acceptance test, common random numbers as the paper's comparison
    W_ind = wl.config_schlogl(args.n_traj)
    W_ind.seed = W.seed + 1000
    ind = ssa.ssa_ensemble_run(items, W_ind.t_end, W_ind.snap_t, W_ind.seed, args.mode, max_events=W.max_events)
    x_ind = ind.snapshots(0)[-1, 0]
    fid_ind = stats.compare(ref_res["x_end"], x_ind)
    fid_crn = stats.compare(ref_res["x_end"], main_res["x_end"])

    # roofline: VALU slots of one event (every-event path of this kernel's code object)
    def per_event(mode):
        f = ssa.ssa_kernel_file(items, W.t_end, W.snap_t, mode)
        return valu_count.count(f)

    ve = per_event(args.mode)
    ve_ref = per_event(args.ref_mode)
    ms = main_res["kernel_ms_avg"]
    achieved = main_res["events_per_step"] * ve["valu_slots"] / (ms * 1e-3)
    value = main_res["events"] / main_res["wall_s"]
    ref_value = ref_res["events"] / ref_res["wall_s"]

    out = {
        "metric": "SSA events/s/GPU: FP16-SR mixed vs FP64 direct, at KS p>0.05 vs oracle",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["wall_s"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16(SR)+f32" if args.mode == "MIX_F16_SR" else args.mode,
        "data": "synthetic",
        "config": {"workload": f"schlogl bistable, {W.n_traj} trajectories, X0=250, T_end=10, 101 snapshots, "
                               f"seed {W.seed}", "mode": args.mode, "ref_mode": args.ref_mode,
                   "events_per_step": main_res["events_per_step"]},
        "fp64": {"value": ref_value, "unit": "events/s", "ms_per_step": ref_res["wall_s"] / args.steps * 1e3,
                 "kernel_ms": ref_res["kernel_ms_avg"], "events_per_step": ref_res["events_per_step"],
                 "valu_slots_per_event": ve_ref["valu_slots"],
                 "valu_frac": ref_res["events_per_step"] * ve_ref["valu_slots"] / (ref_res["kernel_ms_avg"] * 1e-3)
                 / PEAK_VALU_SLOTS},
        "speedup_vs_fp64": value / ref_value,
        "fidelity": {"independent_seeds": fid_ind, "common_random_numbers": fid_crn,
                     "ks_pass": bool(fid_ind["ks_p"] > 0.05)},
        "status_counts": main_res["status_counts"],
        "launch": {k: main_res["info"][k] for k in ("block_size", "grid_size", "vgprs", "n_launches")},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_SLOTS / 1e12,
                     "unit": "TVALU-slot/s", "frac": achieved / PEAK_VALU_SLOTS, "traffic": None,
                     "kernel": "ssa_kernel", "kernel_ms": ms, "valu_slots_per_event": ve["valu_slots"],
                     "valu_insts_per_event": ve["valu_insts"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W, args.mode, args.cpu_sample, log)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
