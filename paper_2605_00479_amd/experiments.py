"""The paper's fidelity experiments on the GPU path.

Each experiment is one of the paper's parameterisations (Sec. 4.1-4.5) run in
FP64 and in the precision configurations of its tables (mixed: FP32, FP16 and
BF16 with RTN or SR; uniform: FP16 and BF16 with RTN or SR, plus this build's
selective-SR and normalised variants). Each reduced-precision ensemble is
compared with the FP64 one at T_end on the marginal the paper reports: KS
statistic and p-value, W1, mean and variance, both with independent seeds
(acceptance) and with common random numbers (the paper's own comparison).

    python -m paper_2605_00479_amd.experiments [--only NAME] [--scale 1.0]

Horizons the paper leaves unstated are chosen long enough for the marginal to
be stationary (noted per experiment).

Three further studies of the paper run as workloads of their own:
  dwell      - the telegraph promoter's OFF / ON dwell times from the event
               record, against the exponential law (Sec. 4.3, telegraph
               validation figure, panel a);
  kon_sweep  - uniform-mode W1 to FP64 across k_on in [1e-3, 1e-1], all k_on
               values in one launch as parameter sets (same figure, panel b);
  horizon    - the repressilator at t_end = 100, 200, 400, 800 from one run
               with snapshots at those times (repressilator horizon figure).
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from dataclasses import dataclass

import numpy as np

from . import stats, workloads as wl

MIXED = ("FP32", "MIX_F16_RTN", "MIX_F16_SR", "MIX_BF16_RTN", "MIX_BF16_SR")
UNIFORM = ("UNI_F16_RTN", "UNI_F16_SR", "UNI_BF16_RTN", "UNI_BF16_SR")
EXTRA = ("UNI_F16_SRA", "UNI_BF16_SRA", "UNI_F16_SR_NORM", "UNI_BF16_SR_NORM")


def schlogl_with_reservoirs(c1=3e-7, c2=1e-4, c3=1e-3, c4=3.5, A=100_000, B=200_000) -> wl.ModelSpec:
    """The paper's original Schloegl parameterisation (Sec. 4.2): the reservoirs
    A and B are species with fixed counts that enter the propensities, so
    A = 1e5 must itself be represented in the propensity type (fp16 cannot)."""
    return wl._build("schlogl_reservoirs", ["X", "A", "B"], [
        {"reactants": {"X": 2, "A": 1}, "change": {"X": +1}, "k": c1},   # (c1/2!) X(X-1) A
        {"reactants": {"X": 3}, "change": {"X": -1}, "k": c2},
        {"reactants": {"B": 1}, "change": {"X": +1}, "k": c3},
        {"reactants": {"X": 1}, "change": {"X": -1}, "k": c4},
    ])


@dataclass
class Experiment:
    name: str
    where: str            # the paper's table
    model: wl.ModelSpec
    x0: tuple
    n_traj: int
    t_end: float
    species: tuple        # marginals reported
    modes: tuple
    max_events: int
    note: str = ""


def experiments(scale: float = 1.0):
    n = lambda k: max(64, int(k * scale))  # noqa: E731
    all_modes = MIXED + UNIFORM + EXTRA
    return {
        "birth_death": Experiment("birth_death", "Table tab:birth-death", wl.birth_death(20.0, 1.0), (0,), n(50_000),
                                  20.0, (0,), all_modes, 200_000, "T_end unstated; 20 relaxation times"),
        "schlogl_original": Experiment("schlogl_original", "Table tab:schlogl", schlogl_with_reservoirs(),
                                       (250, 100_000, 200_000), n(10_000), 10.0, (0,), all_modes, 3_000_000),
        "schlogl_rescaled": Experiment("schlogl_rescaled", "Table tab:schlogl-rescaled", wl.schlogl(), (250,),
                                       n(10_000), 10.0, (0,), all_modes, 3_000_000, "reservoirs folded into k"),
        "telegraph_bimodal": Experiment("telegraph_bimodal", "Table tab:telegraph-bimodal",
                                        wl.telegraph(0.05, 0.05, 20.0, 1.0), (1, 0, 0), n(50_000), 200.0, (2,),
                                        all_modes, 500_000, "T_end unstated; 20 switching times"),
        "telegraph_stress": Experiment("telegraph_stress", "Table tab:telegraph", wl.telegraph(0.01, 0.1, 5.0, 1.0),
                                       (1, 0, 0), n(50_000), 200.0, (2,), all_modes, 200_000,
                                       "T_end unstated; 22 switching times"),
        "dimer": Experiment("dimer", "Table tab:dimer", wl.dimer_closed(1e-3, 0.1), (100, 0), n(50_000), 100.0,
                            (0, 1), all_modes, 500_000, "T_end unstated; stationary by T = 100"),
        "repressilator": Experiment("repressilator", "Table tab:repressilator",
                                    wl.repressilator(alpha0=1.0, alpha=216.0, K=1.0, h=2, dm=1.0, beta=5.0, dp=1.0),
                                    (0, 0, 0, 5, 0, 0), n(10_000), 200.0, (3,), all_modes, 5_000_000),
    }


def prepare_experiment(ex: Experiment):
    """Compile and cache every kernel the experiment launches (no GPU needed)."""
    from . import ssa
    item = [{"model": ssa.Model(ex.model), "x0": np.asarray(ex.x0, np.int32), "n_traj": ex.n_traj}]
    for mode in ("FP64",) + tuple(ex.modes):
        ssa.ssa_prepare(item, ex.t_end, [ex.t_end], mode, max_events=ex.max_events)


def _ensemble(item, t_end, snap_t, seed, mode, max_events):
    from . import ssa
    r = ssa.ssa_ensemble_run([item], t_end, snap_t, seed, mode, max_events=max_events)
    return r


def dwell_times(t, j, n, start_before, on_j=0, off_j=1):
    """OFF dwells (an OFF switch to the next ON switch) and ON dwells from an
    event record, pooled over trajectories, counting only dwells that start
    before ``start_before`` (one still running at the horizon is not in the
    record, so the cut keeps long dwells from being under-represented)."""
    off, on = [], []
    for i in range(n.size):
        k = min(int(n[i]), t.shape[1])
        ti, ji = t[i, :k], j[i, :k]
        start = ti[:-1]
        keep = start < start_before
        d = np.diff(ti)[keep]
        a, b = ji[:-1][keep], ji[1:][keep]
        off.append(d[(a == off_j) & (b == on_j)])
        on.append(d[(a == on_j) & (b == off_j)])
    return np.concatenate(off) if off else np.zeros(0), np.concatenate(on) if on else np.zeros(0)


def dwell_study(scale=1.0, seed=1, log=print):
    """Dwell times of the bimodal telegraph promoter (k_on = k_off = 0.05), so
    OFF and ON dwells are both Exp(0.05) (Sec. 4.3)."""
    from scipy import stats as sst

    from . import ssa
    k_on = k_off = 0.05
    spec = wl.telegraph(k_on, k_off, 20.0, 1.0)
    n = max(64, int(20_000 * scale))
    t_end, cut, cap = 1000.0, 600.0, 96
    item = {"model": ssa.Model(spec), "x0": np.array([1, 0, 0], np.int32), "n_traj": n, "record": (0b11, cap)}
    rows, ref_off = [], None
    for mode in ("FP64",) + MIXED + UNIFORM:
        r = _ensemble(item, t_end, [t_end], seed if mode == "FP64" else seed + 1000, mode, 2_000_000)
        rec = r.records(0)
        if (rec["n"] > cap).any():
            log(f"[dwell] {mode}: {(rec['n'] > cap).sum()} trajectories exceeded the record capacity")
        off, on = dwell_times(rec["t"], rec["j"], rec["n"], cut)
        # quantiles of Exp(k): ln 2 / k (median) and ln 10 / k (90%); in uniform
        # modes dwell times are differences of 16-bit clock values and lie on a
        # lattice, which a KS test against the continuous law detects even
        # when mean and quantiles are right
        row = {"mode": mode, "n_off": int(off.size), "mean_off": float(off.mean()), "mean_on": float(on.mean()),
               "median_off": float(np.median(off)), "q90_off": float(np.quantile(off, 0.9)),
               "ks_p_off_exp": float(sst.kstest(off, "expon", args=(0, 1 / k_on)).pvalue),
               "ks_p_on_exp": float(sst.kstest(on, "expon", args=(0, 1 / k_off)).pvalue)}
        if mode == "FP64":
            ref_off = off
        else:
            row["ks_p_off_vs_fp64"] = float(sst.ks_2samp(off, ref_off).pvalue)
        rows.append(row)
        log(f"[dwell] {mode}: " + ", ".join(f"{k}={v:.4g}" if isinstance(v, float) else f"{k}={v}"
                                           for k, v in row.items() if k != "mode"))
    return rows


def kon_sweep(scale=1.0, seed=1, log=print):
    """Uniform-mode W1 (mRNA at t_end) to FP64 across k_on in [1e-3, 1e-1],
    the other rates of the underflow-stress parameterisation (k_off = 0.1,
    k_m = 5, beta = 1); every k_on is a parameter set of one launch."""
    from . import ssa
    kons = np.logspace(-3, -1, 9)
    per = max(64, int(20_000 * scale))
    spec = wl.telegraph(0.01, 0.1, 5.0, 1.0)
    rates = np.array([[k, 0.1, 5.0, 1.0] for k in kons], np.float64)
    item = {"model": ssa.Model(spec), "x0": np.array([1, 0, 0], np.int32), "n_traj": per * kons.size,
            "set_rates": rates, "traj_per_set": per}
    t_end = 400.0

    def marg(mode, s):
        r = _ensemble(item, t_end, [t_end], s, mode, 2_000_000)
        return r.snapshots(0)[0, 2].reshape(kons.size, per), r.stats(0)["status"].reshape(kons.size, per)

    ref, _ = marg("FP64", seed)
    rows = []
    for mode in ("UNI_F16_RTN", "UNI_F16_SR", "UNI_BF16_RTN", "UNI_BF16_SR", "MIX_BF16_RTN", "MIX_BF16_SR"):
        m, st = marg(mode, seed + 1000)
        row = {"mode": mode}
        for i, k in enumerate(kons):
            c = stats.compare(ref[i], m[i])
            row[f"{k:.3g}"] = {"w1": c["w1"], "ks_p": c["ks_p"], "mean": c["mean"], "mean_ref": c["mean_ref"],
                               "capped": int((st[i] == 3).sum())}
        rows.append(row)
        log(f"[kon_sweep] {mode}: W1 " + ", ".join(f"{k}:{v['w1']:.3g}" for k, v in row.items() if k != "mode"))
    return {"k_on": kons.tolist(), "per_set": per, "t_end": t_end, "rows": rows}


def horizon_sweep(scale=1.0, seed=1, log=print):
    """The repressilator's p_0 marginal at t_end = 100, 200, 400, 800 under
    uniform precision, from one run per mode with snapshots at those times
    (each snapshot equals the end state of a run stopped there)."""
    from . import ssa
    spec = wl.repressilator(alpha0=1.0, alpha=216.0, K=1.0, h=2, dm=1.0, beta=5.0, dp=1.0)
    n = max(64, int(10_000 * scale))
    hs = [100.0, 200.0, 400.0, 800.0]
    item = {"model": ssa.Model(spec), "x0": np.array([0, 0, 0, 5, 0, 0], np.int32), "n_traj": n}
    ref = _ensemble(item, hs[-1], hs, seed, "FP64", 20_000_000).snapshots(0)[:, 3]
    rows = []
    for mode in ("UNI_F16_SR", "UNI_BF16_SR", "UNI_F16_SR_NORM", "UNI_BF16_SR_NORM", "MIX_F16_SR", "MIX_BF16_SR"):
        r = _ensemble(item, hs[-1], hs, seed + 1000, mode, 20_000_000)
        snap, st = r.snapshots(0)[:, 3], r.stats(0)["status"]
        row = {"mode": mode, "capped": int((st == 3).sum())}
        for k, h in enumerate(hs):
            c = stats.compare(ref[k], snap[k])
            row[f"{h:g}"] = {"w1": c["w1"], "ks_p": c["ks_p"], "mean": c["mean"], "mean_ref": c["mean_ref"]}
        rows.append(row)
        log(f"[horizon] {mode}: " + ", ".join(f"t={h:g} W1={row[f'{h:g}']['w1']:.3g} p={row[f'{h:g}']['ks_p']:.3g}"
                                             for h in hs))
    return {"horizons": hs, "n": n, "rows": rows}


def run_experiment(ex: Experiment, seed: int = 1, log=print):
    from . import ssa
    model = ssa.Model(ex.model)
    item = [{"model": model, "x0": np.asarray(ex.x0, np.int32), "n_traj": ex.n_traj}]
    ts = [ex.t_end]

    def go(mode, s):
        t0 = time.perf_counter()
        r = ssa.ssa_ensemble_run(item, ex.t_end, ts, s, mode, max_events=ex.max_events)
        snap, st = r.snapshots(0), r.stats(0)
        info = r.info()
        return snap[0], st, info, time.perf_counter() - t0

    ref, ref_st, ref_info, _ = go("FP64", seed)
    rows = [{"mode": "FP64", "events_per_s": ref_info["total_events"] / (ref_info["elapsed_ms"] * 1e-3),
             **{f"mean_{s}": float(ref[s].mean()) for s in ex.species},
             **{f"var_{s}": float(ref[s].var(ddof=1)) for s in ex.species}}]
    for mode in ex.modes:
        crn, st, info, _ = go(mode, seed)
        ind, st_ind, _, _ = go(mode, seed + 1000)
        row = {"mode": mode, "events_per_s": info["total_events"] / (info["elapsed_ms"] * 1e-3),
               "status": np.bincount(st["status"], minlength=4).tolist()}
        for s in ex.species:
            ci = stats.compare(ref[s], ind[s])
            cc = stats.compare(ref[s], crn[s])
            row.update({f"ks_p_{s}": ci["ks_p"], f"w1_{s}": ci["w1"], f"mean_{s}": ci["mean"], f"var_{s}": ci["var"],
                        f"ks_p_crn_{s}": cc["ks_p"], f"w1_crn_{s}": cc["w1"]})
        rows.append(row)
        log(f"[{ex.name}] {mode}: " + ", ".join(f"{k}={v:.4g}" if isinstance(v, float) else f"{k}={v}"
                                               for k, v in row.items() if k != "mode"))
    return rows


def to_markdown(ex: Experiment, rows) -> str:
    sp = [ex.model.species[s] for s in ex.species]
    head = "| mode | " + " | ".join(f"KS p ({n}) | W1 ({n}) | mean ({n}) | var ({n}) | KS p CRN ({n})" for n in sp) + \
           " | overflow / capped | events/s |"
    lines = [f"**{ex.name}** ({ex.where}; {ex.n_traj} trajectories, T_end {ex.t_end}{'; ' + ex.note if ex.note else ''})",
             "", head, "|" + "---|" * (2 + 5 * len(sp) + 1)]
    for r in rows:
        cells = []
        for s in ex.species:
            if r["mode"] == "FP64":
                cells += ["—", "—", f"{r[f'mean_{s}']:.4g}", f"{r[f'var_{s}']:.4g}", "—"]
            else:
                cells += [f"{r[f'ks_p_{s}']:.3g}", f"{r[f'w1_{s}']:.3g}", f"{r[f'mean_{s}']:.4g}",
                          f"{r[f'var_{s}']:.4g}", f"{r[f'ks_p_crn_{s}']:.3g}"]
        st = r.get("status", [0, 0, 0, 0])
        lines.append(f"| {r['mode']} | " + " | ".join(cells) + f" | {st[2]} / {st[3]} | {r['events_per_s']:.3g} |")
    return "\n".join(lines)


def main(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--only", default=None)
    p.add_argument("--scale", type=float, default=1.0)
    p.add_argument("--json", default=None)
    p.add_argument("--prepare", action="store_true", help="only compile the kernels (no GPU needed)")
    p.add_argument("--studies", default="", help="comma-separated: dwell, kon_sweep, horizon (instead of the tables)")
    a = p.parse_args(argv)
    if a.studies:
        log = (lambda m: print(m, file=sys.stderr, flush=True))
        fns = {"dwell": dwell_study, "kon_sweep": kon_sweep, "horizon": horizon_sweep}
        out = {name: fns[name](a.scale, log=log) for name in a.studies.split(",")}
        print(json.dumps(out, indent=1))
        if a.json:
            with open(a.json, "w") as f:
                json.dump(out, f)
        return
    exs = experiments(a.scale)
    names = [a.only] if a.only else list(exs)
    if a.prepare:
        for name in names:
            prepare_experiment(exs[name])
        return
    out = {}
    for name in names:
        rows = run_experiment(exs[name], log=lambda m: print(m, file=sys.stderr, flush=True))
        out[name] = rows
        print(to_markdown(exs[name], rows), flush=True)
        print(flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(out, f)


if __name__ == "__main__":
    main()
