"""GPU path vs oracle on the paper's own parameterisations and sweeps, through
the C ABI, trajectory by trajectory (same bar as test_gpu_parity.py: counts,
event counts and statuses bit-exact, the last event's time within 1e-12
relative in FP64 and 1e-6 with binary32 or 16-bit clocks).

* the k_on sweep of the telegraph validation figure (Sec. 4.3, panel b): nine
  k_on values as per-lane parameter sets of one launch;
* the repressilator of Sec. 4.5 (Table tab:repressilator parameters) with
  snapshots at the horizons of the repressilator drift figure;
* the original Schloegl parameterisation with reservoir species (Sec. 4.2,
  Table tab:schlogl): fp16 cannot hold A = 1e5, bf16 can;
* the closed dimerisation 2A <-> D (Sec. 4.4, Table tab:dimer) in uniform
  stochastic rounding, where A + 2D must stay exact.
"""
import numpy as np
import pytest

from paper_2605_00479_amd import experiments as ex
from paper_2605_00479_amd import workloads as wl

pytestmark = pytest.mark.gpu

ORACLE_THREADS = 16


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_2605_00479_amd import ssa
    ssa.lib()
    return ssa


def assert_parity(ref, snap, st, mode, label):
    np.testing.assert_array_equal(snap, ref["snap"], err_msg=f"snapshots {label} {mode}")
    np.testing.assert_array_equal(st["status"], ref["status"], err_msg=f"status {label} {mode}")
    np.testing.assert_array_equal(st["n_events"], ref["n_events"], err_msg=f"events {label} {mode}")
    a, b = st["t_last"], ref["t_last"]
    tol = 1e-12 if mode == "FP64" else 1e-6
    rel = np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
    assert np.all((a == b) | (rel <= tol)), f"t_last {label} {mode}: max rel {rel.max()}"


def run_both(gpu, orc, spec, x0, n, t_end, snap_t, mode, *, seed, max_events, set_rate=None, traj_per_set=0,
             **launch):
    item = {"model": gpu.Model(spec), "x0": np.asarray(x0, np.int32), "n_traj": n}
    if set_rate is not None:
        item["set_rates"] = set_rate
        item["traj_per_set"] = traj_per_set
    print(f"[gpu-paper] {spec.name} mode={mode} n={n} t_end={t_end} launch={launch}", flush=True)
    run = gpu.ssa_ensemble_run([item], t_end, snap_t, seed, mode, max_events=max_events, **launch)
    snap, st = run.snapshots(0), run.stats(0)
    ref = orc.simulate(spec, mode, np.asarray(x0, np.int32), t_end, np.asarray(snap_t, float), seed, n_traj=n,
                       max_events=max_events, set_rate=set_rate, traj_per_set=traj_per_set, threads=ORACLE_THREADS)
    assert_parity(ref, snap, st, mode, spec.name)
    return snap, st


@pytest.mark.parametrize("mode,cap", [("UNI_F16_SR", 200_000), ("UNI_BF16_RTN", 20_000), ("FP64", 200_000),
                                      ("MIX_BF16_SR", 200_000)])
def test_kon_sweep_parameter_sets(gpu, orc, mode, cap):
    """k_on in [1e-3, 1e-1] (nine log-spaced values), k_off = 0.1, k_m = 5,
    beta = 1, T = 400: every k_on is a parameter set of one launch, 40
    trajectories each. Uniform bf16 round to nearest runs with a cap (its
    clock can stall; at these rates none of these trajectories reaches it)."""
    kons = np.logspace(-3, -1, 9)
    rates = np.array([[k, 0.1, 5.0, 1.0] for k in kons], np.float64)
    spec = wl.telegraph(0.01, 0.1, 5.0, 1.0)
    snap, st = run_both(gpu, orc, spec, [1, 0, 0], 9 * 40, 400.0, [100.0, 400.0], mode, seed=21, max_events=cap,
                        set_rate=rates, traj_per_set=40)
    # gene copies are conserved exactly in every mode
    assert np.all(snap[:, 0, :] + snap[:, 1, :] == 1)


@pytest.mark.parametrize("mode,launch", [("UNI_BF16_SR", {}), ("UNI_F16_SR_NORM", {}), ("MIX_F16_SR", {}),
                                         ("FP64", {}), ("UNI_BF16_SR", {"block_size": 512})])
def test_paper_repressilator_horizons(gpu, orc, mode, launch):
    """The paper's repressilator (alpha0 = 1, alpha = 216, K = 1, h = 2,
    mRNA decay 1, translation 5, protein decay 1; p = (5, 0, 0)) to T = 800
    with snapshots at t = 100, 200, 400, 800 (each the end state of a run
    stopped there): about 3e5 events per trajectory."""
    e = ex.experiments()["repressilator"]
    run_both(gpu, orc, e.model, e.x0, 128, 800.0, [100.0, 200.0, 400.0, 800.0], mode, seed=23,
             max_events=20_000_000, **launch)


@pytest.mark.parametrize("mode", ["MIX_F16_SR", "MIX_F16_RTN", "MIX_BF16_SR", "UNI_BF16_SR", "FP64"])
def test_schlogl_with_reservoir_species(gpu, orc, mode):
    """Schloegl with A = 1e5 and B = 2e5 as species (Table tab:schlogl). In
    fp16 the count A converts to infinity, so every trajectory overflows at
    its first event with X frozen at 250; bf16 holds A and runs on."""
    e = ex.experiments()["schlogl_original"]
    snap, st = run_both(gpu, orc, e.model, e.x0, 400, 10.0, wl.snapshot_grid(10.0, 11), mode, seed=25,
                        max_events=e.max_events)
    if mode.startswith("MIX_F16"):
        assert np.all(st["status"] == 2) and np.all(st["n_events"] == 0) and np.all(snap[:, 0, :] == 250)
    else:
        assert np.all(st["status"] == 0)
    # the reservoir counts never change
    assert np.all(snap[:, 1, :] == 100_000) and np.all(snap[:, 2, :] == 200_000)


@pytest.mark.parametrize("mode", ["UNI_F16_SR", "UNI_BF16_SR", "UNI_BF16_SR_NORM", "UNI_F16_SRA"])
def test_closed_dimer_uniform_sr(gpu, orc, mode):
    """2A <-> D with kf = 1e-3, kr = 0.1 from A = 100 (Table tab:dimer), in
    uniform 16-bit modes: A + 2D = 100 in every snapshot of every trajectory."""
    e = ex.experiments()["dimer"]
    snap, _ = run_both(gpu, orc, e.model, e.x0, 2000, 100.0, wl.snapshot_grid(100.0, 11), mode, seed=27,
                       max_events=e.max_events)
    assert np.all(snap[:, 0, :] + 2 * snap[:, 1, :] == 100)
