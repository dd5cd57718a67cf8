"""Benchmark: SSA events/s on one MI355X, mixed FP16 with stochastic rounding
(the reported value) against the FP64 direct method, on the open-dimerisation
parameter sweep in one persistent launch (4,096 log-uniform parameter sets x
256 trajectories, T_end = 50, 51 snapshots) unless --config names another
configured workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config dimer_sweep]

A step is one complete ensemble run (every trajectory from t = 0 to T_end:
RNG draws, propensities, sums, waiting times, snapshot stores, selection and
integer updates) through the C ABI. Prints one JSON line. `value` counts only
when the reduced-precision end-time marginals pass KS (p > 0.05, independent
seeds) against the FP64 ensemble; otherwise it is null and the measured rate
is reported as `value_failing_fidelity`.
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

# species whose end-time marginal the fidelity statistics use, per network
MARGINALS = {"birth_death": (0,), "schlogl": (0,), "telegraph": (2,), "dimer_open": (0, 1),
             "repressilator": (3,), "dimer_closed": (0, 1)}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--config", default="dimer_sweep")
    p.add_argument("--n-traj", type=int, default=0, help="override the ensemble size (0: the config's)")
    p.add_argument("--mode", default="MIX_F16_SR")
    p.add_argument("--ref-mode", default="FP64")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fidelity", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=16000, help="trajectories the oracle runs for cpu_baseline")
    p.add_argument("--chunks", type=int, default=0, help="0: autotuned (or 1 without --no-autotune's tuning)")
    p.add_argument("--no-autotune", action="store_true")
    p.add_argument("--valu-peak", action="store_true", help="also measure per-class VALU rates")
    p.add_argument("--copy-calib", action="store_true",
                   help="also run a 1 GiB device copy (calibrates the profiler's memory counters)")
    p.add_argument("--block", type=int, default=0)
    p.add_argument("--grid", type=int, default=0)
    p.add_argument("--first-window", type=int, default=0)
    p.add_argument("--placement", type=int, default=0,
                   help="0: autotuned; else 1 | 2 (producer on the next SIMD) | 4 (wave-major first claims)")
    return p.parse_args()


def make_workload(name, n):
    from paper_2605_00479_amd import workloads as wl
    make = wl.CONFIGS[name]
    if not n:
        return make()
    if name == "dimer_sweep":
        return make(n_sets=max(1, n // 256))
    if name == "heterogeneous":
        return make(n_traj_total=n)
    return make(n)


def launch(ssa, items, W, mode, seed, args):
    return ssa.ssa_ensemble_run(items, W.t_end, W.snap_t, seed, mode, max_events=W.max_events,
                                n_chunks=args.chunks, block_size=args.block, grid_size=args.grid,
                                first_window=args.first_window, placement=args.placement)


def marginals(run, W):
    """End-time rows of the marginal species, taken from the run's device
    output tensors (only these rows cross to the host)."""
    out = {}
    for i, it in enumerate(W.items):
        snap = run.tensors(i)[0]
        for s in MARGINALS.get(it.model.name, (0,)):
            out[f"{it.model.name}:{it.model.species[s]}"] = (snap[-1, s].cpu().numpy().copy() if snap.shape[0]
                                                            else np.zeros(0))
    return out


def timed_runs(ssa, items, W, mode, args, log):
    import torch
    if not args.no_autotune and not (args.block or args.grid or args.chunks):
        tuned = ssa.ssa_autotune(items, W.t_end, W.snap_t, W.seed, mode, max_events=W.max_events)
        log(f"[bench] autotune {mode}: {tuned}")
    for _ in range(args.warmup):
        launch(ssa, items, W, mode, W.seed, args).wait()
    torch.cuda.synchronize()
    runs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        runs.append(launch(ssa, items, W, mode, W.seed, args))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    infos = [r.info() for r in runs]
    events = sum(i["total_events"] for i in infos)
    kern_ms = [i["kernel_ms"] for i in infos]
    log(f"[bench] {mode}: {args.steps} steps, {events} events, wall {wall:.3f}s, kernel ms {kern_ms}")
    last = runs[-1]
    status = np.zeros(4, dtype=np.int64)
    item_events = []
    max_events = 0
    for i in range(len(W.items)):
        st = last.stats(i)
        status += np.bincount(st["status"], minlength=4)[:4]
        item_events.append(float(st["n_events"].sum()))
        if st["n_events"].size:
            max_events = max(max_events, int(st["n_events"].max()))
    return {"wall_s": wall, "events": events, "events_per_step": events / args.steps,
            "kernel_ms_avg": float(np.mean(kern_ms)), "info": infos[-1],
            "marg": None if args.no_fidelity else marginals(last, W), "status_counts": status.tolist(),
            "item_events": item_events, "max_events": max_events}


VALU_CLASSES = ["v_add_u32", "v_bitop3_b32", "v_mad_u64_u32", "v_mul_f32", "v_fma_f32", "v_mul_f64", "v_fma_f64",
                "v_rcp_f32", "v_rcp_f64", "v_cvt_sr_f16_f32 + v_cvt_f32_f16", "v_cvt_f16_f32 + v_cvt_f32_f16",
                "v_add_f32", "v_add_f64", "v_cvt_f32_i32 + v_cvt_i32_f32", "v_mul_hi_u32 + v_or_b32", "v_cndmask_b32",
                "v_add_f32 (VGPR operands)"]
# (waves per SIMD, independent chains per lane): SIMD throughput, one wave's issue, dependent latency
VALU_SHAPES = {"throughput_8w8c": (8, 8), "one_wave_8c": (1, 8), "latency_1w1c": (1, 1)}


def valu_peak(log):
    """Measured issue cost per instruction class: SIMD cycles per wave64 step
    at the nominal 2.4 GHz (4 = one full-rate wave64 instruction on a SIMD16)."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2605_00479_amd", "libssa_valu_peak.so"))
    lib.valu_peak_run_shape.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    if lib.valu_peak_count() != len(VALU_CLASSES):
        raise RuntimeError("libssa_valu_peak.so does not match bench.py's class list")
    simd_lane_cycles = 256 * 4 * 2.4e9 * 64
    out = []
    for op, name in enumerate(VALU_CLASSES):
        row = {"class": name}
        for shape, (w, c) in VALU_SHAPES.items():
            rate, ms = ctypes.c_double(), ctypes.c_double()
            iters = 256 if w == 8 else 1024
            if lib.valu_peak_run_shape(op, iters, w, c, ctypes.byref(rate), ctypes.byref(ms)) != 0:
                raise RuntimeError("valu_peak_run_shape failed")
            row[shape] = simd_lane_cycles / rate.value
        out.append(row)
        log(f"[bench] valu {name}: cycles/wave64 step " +
            ", ".join(f"{k} {row[k]:.2f}" for k in VALU_SHAPES))
    return out


def copy_calib(log, nbytes=1 << 30):
    """One plain device-to-device copy of nbytes (kernel hbm_copy_kernel)."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2605_00479_amd", "libssa_valu_peak.so"))
    lib.hbm_copy_run.argtypes = [ctypes.c_size_t, ctypes.POINTER(ctypes.c_double)]
    ms = ctypes.c_double()
    if lib.hbm_copy_run(nbytes, ctypes.byref(ms)) != 0:
        raise RuntimeError("hbm_copy_run failed")
    gbs = 2 * nbytes / (ms.value * 1e-3) / 1e9
    log(f"[bench] copy {nbytes} B: {ms.value:.3f} ms = {gbs:.0f} GB/s (read + write)")
    return {"bytes": nbytes, "ms": ms.value, "GB_per_s_read_plus_write": gbs}


TRAFFIC_FILES = {"schlogl": "ssa_kernel_schlogl_100k_traffic.md",
                 "dimer_sweep": "ssa_kernel_dimer_sweep_traffic.md"}


def measured_traffic(workload, mode, kernel_file):
    """HBM bytes per step from the committed counter summary of the workload,
    if it was taken on this exact kernel object (rows: | mode | object | ... |
    bytes |)."""
    name = TRAFFIC_FILES.get(workload)
    path = os.path.join(ROOT, "profiles", name) if name else None
    if not path or not os.path.exists(path):
        return None
    obj = os.path.basename(kernel_file)
    for line in open(path):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 3 and cells[0] == mode and cells[1] == obj:
            try:
                return float(cells[-1])
            except ValueError:
                return None
    return None


def physical_cores():
    """Distinct (package, core) pairs among the CPUs this process may run on."""
    try:
        allowed = os.sched_getaffinity(0)
        pairs, cpu, phys = set(), None, None
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "processor":
                    cpu = int(v)
                elif k == "physical id":
                    phys = v
                elif k == "core id" and cpu in allowed:
                    pairs.add((phys, v))
        return len(pairs) or None
    except (OSError, ValueError):
        return None


def cpu_baseline(W, mode, n_sample, log):
    """The oracle on the host's cores, on every k-th trajectory of the same
    ensemble (k = E / n_sample, so the sample spans every parameter set)."""
    import oracle
    allowed = len(os.sched_getaffinity(0))
    threads = min(16, allowed)
    it = W.items[0]
    n = min(n_sample, it.n_traj)
    stride = max(1, it.n_traj // n)
    idx = np.arange(0, stride * n, stride, dtype=np.int64)
    t0 = time.perf_counter()
    r = oracle.simulate(it.model, mode, it.x0, W.t_end, W.snap_t, W.seed, indices=idx, max_events=W.max_events,
                        set_rate=it.set_rate, traj_per_set=it.traj_per_set, threads=threads)
    dt = time.perf_counter() - t0
    ev = int(r["n_events"].sum())
    log(f"[bench] cpu oracle {mode}: {n} trajectories, {ev} events in {dt:.2f}s on {threads} threads")
    return {"value": ev / dt, "unit": "events/s", "cores": threads, "physical_cores": physical_cores(),
            "cpus_available": allowed, "kind": "oracle",
            "sample": f"every {stride}th trajectory (ids 0, {stride}, ..., {int(idx[-1])}; {n} in all) of the same "
                      f"{it.model.name} ensemble, {mode}, full horizon, {ev} events"}


def main():
    args = parse()
    log = (lambda m: print(m, file=sys.stderr, flush=True))
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the path has no multi-GPU part); got --gpus {args.gpus}",
              file=sys.stderr)
        return 2
    import torch
    from paper_2605_00479_amd import ssa, stats
    from paper_2605_00479_amd.csrc import valu_count
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    ssa.lib()
    W = make_workload(args.config, args.n_traj)
    items = ssa.items_from_workload(W)
    log(f"[bench] workload {W.name}: {W.n_traj} trajectories, T_end {W.t_end}, {len(W.snap_t)} snapshots")

    main_res = timed_runs(ssa, items, W, args.mode, args, log)
    ref_res = timed_runs(ssa, items, W, args.ref_mode, args, log)

    fidelity = None
    if not args.no_fidelity:
        # end-time marginals against FP64: independent seeds (acceptance) and common random numbers
        ind = launch(ssa, items, W, args.mode, W.seed + 1000, args)
        m_ind = marginals(ind, W)
        fidelity = {}
        for key, ref in ref_res["marg"].items():
            fidelity[key] = {"independent_seeds": stats.compare(ref, m_ind[key]),
                             "common_random_numbers": stats.compare(ref, main_res["marg"][key])}
        fails = [k for k, v in fidelity.items() if v["independent_seeds"]["ks_p"] <= 0.05]
        fidelity["ks_pass_all"] = not fails
        fidelity["ks_fail"] = fails

    # roofline: VALU slots of one event on the every-event path of the launched
    # code object, counted on its one-wave event loop (ssa_kernel). With producer
    # waves (ssa_kernel_pc, 512-thread workgroups) the same per-event work is
    # split between the paired waves; the LDS ring traffic is not counted.
    # Several networks in one launch: the object's lightest loop would understate
    # the work, so each network's slots are counted on its own single-network
    # object and weighted by the events that network fired.
    def per_event(mode, res):
        f = ssa.ssa_kernel_file(items, W.t_end, W.snap_t, mode, max_events=W.max_events)
        c = {**valu_count.count(f), "file": f}
        ev = np.asarray(res["item_events"])
        if len(items) > 1 and ev.sum() > 0:
            per = [valu_count.count(ssa.ssa_kernel_file([it], W.t_end, W.snap_t, mode, max_events=W.max_events))
                   for it in items]
            for key in ("valu_slots", "valu_insts"):
                c[key] = float(sum(e * p[key] for e, p in zip(ev, per)) / ev.sum())
        return c

    ve, ve_ref = per_event(args.mode, main_res), per_event(args.ref_mode, ref_res)
    ms = main_res["kernel_ms_avg"]
    achieved = main_res["events_per_step"] * ve["valu_slots"] / (ms * 1e-3)
    rate = main_res["events"] / main_res["wall_s"]
    # the metric counts events/s only where the ensemble passes KS against FP64
    passed = fidelity is not None and fidelity["ks_pass_all"]
    value = rate if passed else None
    ref_value = ref_res["events"] / ref_res["wall_s"]
    desc = {"schlogl": "schlogl bistable, X0=250, T_end=10, 101 snapshots",
            "birth_death": "birth-death kb=10 kd=0.1, X0=0, T_end=100, snapshot at 100",
            "telegraph": "telegraph k_on=0.05 k_off=0.1 k_m=20, gene off, T_end=200, 201 snapshots",
            "dimer_sweep": "open dimerisation sweep in one launch: 4,096 parameter sets (k1..k4 = 50, 0.1, 0.001, 0.5 "
                           "each x 10^(2u-1), u from PCG64 seed 7) x 256 trajectories, M0=D0=0, T_end=50, 51 snapshots",
            "heterogeneous": "five networks in one launch, T_end=500, 501 snapshots"}[W.name]
    out_cfg_chunks = main_res["info"]["n_launches"]
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
        "config": {"workload": f"{desc}, {W.n_traj} trajectories, seed {W.seed}", "mode": args.mode,
                   "ref_mode": args.ref_mode, "events_per_step": main_res["events_per_step"],
                   "n_chunks": out_cfg_chunks},
        "fp64": {"value": ref_value, "unit": "events/s", "ms_per_step": ref_res["wall_s"] / args.steps * 1e3,
                 "kernel_ms": ref_res["kernel_ms_avg"], "events_per_step": ref_res["events_per_step"],
                 "valu_slots_per_event": ve_ref["valu_slots"],
                 "valu_frac": ref_res["events_per_step"] * ve_ref["valu_slots"] / (ref_res["kernel_ms_avg"] * 1e-3)
                 / PEAK_VALU_SLOTS},
        "speedup_vs_fp64": rate / ref_value,
        "fidelity": fidelity,
        "fidelity_gate": "passed" if passed else ("skipped" if fidelity is None else "failed"),
        "status_counts": main_res["status_counts"],
        "launch": {k: main_res["info"][k] for k in ("block_size", "grid_size", "vgprs", "n_launches", "first_window",
                                                     "placement")},
        "launch_fp64": {k: ref_res["info"][k] for k in ("block_size", "grid_size", "vgprs", "n_launches",
                                                          "first_window", "placement")},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_SLOTS / 1e12,
                     "unit": "TVALU-slot/s", "frac": achieved / PEAK_VALU_SLOTS,
                     "traffic": measured_traffic(W.name, args.mode, ve["file"]),
                     "kernel": "ssa_kernel_pc" if main_res["info"]["block_size"] == 512 else "ssa_kernel",
                     "kernel_object": os.path.basename(ve["file"]), "kernel_ms": ms,
                     "valu_slots_per_event": ve["valu_slots"], "valu_insts_per_event": ve["valu_insts"]},
    }
    # the chain bound: no launch ends before its longest trajectory has fired all
    # its events one after another; cycles per event of that chain at the nominal clock
    out["chain"] = {"max_events_per_trajectory": main_res["max_events"],
                    "cycles_per_event_at_2.4GHz": ms * 1e-3 * 2.4e9 / max(main_res["max_events"], 1),
                    "fp64_max_events_per_trajectory": ref_res["max_events"],
                    "fp64_cycles_per_event_at_2.4GHz":
                        ref_res["kernel_ms_avg"] * 1e-3 * 2.4e9 / max(ref_res["max_events"], 1)}
    if not passed:
        out["value_failing_fidelity"] = rate
    out["fp64"]["kernel_object"] = os.path.basename(ve_ref["file"])
    out["fp64"]["kernel"] = "ssa_kernel_pc" if ref_res["info"]["block_size"] == 512 else "ssa_kernel"
    if args.valu_peak:
        out["valu_peak"] = valu_peak(log)
    if args.copy_calib:
        out["copy_calib"] = copy_calib(log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W, args.mode, args.cpu_sample, log)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
