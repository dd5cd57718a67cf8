"""GPU path vs oracle, trajectory by trajectory, through the C ABI.

The bar: species counts, event counts and statuses bit-exact; the time of the
last event within 1e-12 relative (FP64) or 1e-6 relative (binary32 clocks).
Sizes are chosen so the oracle finishes in seconds while the launch still
spans many waves, ragged tails and the lane-refill path; the full-size
Schloegl ensemble is checked on a sample of trajectory ids.
"""
import numpy as np
import pytest

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


def tol_for(mode):
    return 1e-12 if mode == "FP64" else 1e-6


def assert_parity(orc_res, snap, stats, mode, label=""):
    np.testing.assert_array_equal(snap, orc_res["snap"], err_msg=f"snapshots {label} {mode}")
    np.testing.assert_array_equal(stats["status"], orc_res["status"], err_msg=f"status {label} {mode}")
    np.testing.assert_array_equal(stats["n_events"], orc_res["n_events"], err_msg=f"events {label} {mode}")
    a, b = stats["t_last"], orc_res["t_last"]
    rel = np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
    assert np.all((a == b) | (rel <= tol_for(mode))), f"t_last {label} {mode}: max rel {rel.max()}"


# Event cap of test runs that name none: far above any test trajectory's count
# (a binary32 or 16-bit clock needs a finite cap, the library refuses none)
TEST_CAP = 50_000_000


def run_both(gpu, orc, spec, x0, n, t_end, snap_t, mode, *, seed=1, max_events=0, set_rate=None,
             traj_per_set=0, indices=None, **launch):
    max_events = max_events or TEST_CAP
    m = gpu.Model(spec)
    item = {"model": m, "x0": x0, "n_traj": n}
    if set_rate is not None:
        item["set_rates"] = set_rate
        item["traj_per_set"] = traj_per_set
    print(f"[gpu-parity] {spec.name} mode={mode} n={n} seed={seed} launch={launch}", flush=True)
    run = gpu.ssa_ensemble_run([item], t_end, snap_t, seed, mode, max_events=max_events, **launch)
    snap = run.snapshots(0)
    st = run.stats(0)
    idx = np.arange(n) if indices is None else np.asarray(indices)
    ref = orc.simulate(spec, mode, x0, t_end, snap_t, seed, indices=idx, max_events=max_events,
                       set_rate=set_rate, traj_per_set=traj_per_set, threads=ORACLE_THREADS)
    st = {k: v[idx] for k, v in st.items()}
    assert_parity(ref, snap[:, :, idx], st, mode, spec.name)
    return run, snap, st


def test_birth_death_config_fp64(gpu, orc):
    W = wl.config_birth_death()
    it = W.items[0]
    run_both(gpu, orc, it.model, it.x0, it.n_traj, W.t_end, W.snap_t, "FP64", seed=W.seed)


@pytest.mark.parametrize("mode", ["FP64", "FP32", "MIX_F16_RTN", "MIX_F16_SR", "MIX_BF16_RTN", "MIX_BF16_SR"])
def test_schlogl_modes(gpu, orc, mode):
    W = wl.config_schlogl()
    it = W.items[0]
    run_both(gpu, orc, it.model, it.x0, 1500, W.t_end, W.snap_t, mode, seed=W.seed, max_events=W.max_events)


@pytest.mark.parametrize("mode,cap", [("UNI_F16_SRA", 0), ("UNI_F16_SR", 0), ("UNI_F16_RTN", 100_000),
                                      ("UNI_BF16_SR_NORM", 0)])
def test_schlogl_uniform_modes(gpu, orc, mode, cap):
    """Uniform 16-bit runs of the Schloegl network. Its totals reach several
    thousand, where the selection target (the binary32 product u2 * a0,
    then one rounding to the 16-bit type) meets ties of the second rounding
    (u2 has 24 bits, so rounding the exact product once can differ).
    Round to nearest stalls the clock: capped runs."""
    W = wl.config_schlogl()
    it = W.items[0]
    run_both(gpu, orc, it.model, it.x0, 1500, W.t_end, W.snap_t, mode, seed=W.seed,
             max_events=cap or W.max_events)


@pytest.mark.parametrize("mode", ["UNI_F16_RTN", "UNI_F16_SR", "UNI_F16_SR_NORM", "UNI_BF16_RTN",
                                  "UNI_BF16_SR", "UNI_BF16_SR_NORM", "UNI_F16_RTN_NORM", "FP64",
                                  "UNI_F16_SRA", "UNI_BF16_SRA_NORM"])
def test_telegraph_uniform_modes(gpu, orc, mode):
    W = wl.config_telegraph()
    it = W.items[0]
    run_both(gpu, orc, it.model, it.x0, 1000, 60.0, wl.snapshot_grid(60.0, 61), mode, seed=W.seed,
             max_events=W.max_events)


@pytest.mark.parametrize("mode", ["FP64", "MIX_F16_SR", "MIX_BF16_SR", "UNI_F16_SR", "UNI_BF16_SRA"])
def test_repressilator_hill_laws(gpu, orc, mode):
    m = wl.repressilator()
    run_both(gpu, orc, m, np.array([0, 0, 0, 0, 0, 20], np.int32), 600, 60.0, wl.snapshot_grid(60.0, 61),
             mode, seed=3, max_events=10_000_000)


@pytest.mark.parametrize("mode", ["FP64", "MIX_F16_SR"])
def test_dimer_parameter_sets_per_lane(gpu, orc, mode):
    rates = wl.dimer_sweep_rates(48)
    m = wl.dimer_open()
    run_both(gpu, orc, m, np.array([0, 0], np.int32), 48 * 40, 10.0, wl.snapshot_grid(10.0, 11), mode,
             seed=1, set_rate=rates, traj_per_set=40, max_events=3_000_000)


@pytest.mark.parametrize("mode,levels", [("MIX_F16_SR", (1500.0, 2100.0, 2600.0)),
                                         ("UNI_F16_SR", (1500.0, 2100.0, 2600.0)),
                                         ("MIX_F16_RTN", (1500.0, 2100.0, 2600.0)),
                                         ("MIX_BF16_SR", (180.0, 250.0, 330.0))])
def test_count_conversion_across_exact_integer_limit(gpu, orc, mode, levels):
    # Counts up to 2^11 (fp16) or 2^8 (bf16) convert exactly; above that the
    # conversion itself rounds (by SR or RNE) and draws its rounding slot.
    # Birth-death sets around the limit put lanes of one wave on both sides
    # of it, and counts cross it during the run.
    kd = 1.0
    rates = np.array([[kb, kd] for kb in levels], np.float64)
    start = np.int32(levels[1])
    run_both(gpu, orc, wl.birth_death(levels[1], kd), np.array([start], np.int32), 3 * 70, 1.5,
             wl.snapshot_grid(1.5, 7), mode, seed=11, set_rate=rates, traj_per_set=70, max_events=200_000)


def low_count_network():
    """Two species whose counts sit near the reactant orders (means about 8
    and 12): X + Y -> X and 2X -> X, 3Y -> 2Y. Lanes dip below the orders now
    and then, so a wave moves between the propensity version without zero
    guards (every count at or above its largest order: 2 for X, 3 for Y) and
    the guarded one, and the start (0, 0) is guarded."""
    return wl._build("low_count", ["X", "Y"], [
        {"change": {"X": +1}, "k": 8.0},
        {"reactants": {"X": 1}, "change": {"X": -1}, "k": 1.0},
        {"change": {"Y": +1}, "k": 12.0},
        {"reactants": {"Y": 1}, "change": {"Y": -1}, "k": 1.0},
        {"reactants": {"X": 1, "Y": 1}, "change": {"Y": -1}, "k": 0.02},
        {"reactants": {"X": 2}, "change": {"X": -1}, "k": 0.05},
        {"reactants": {"Y": 3}, "change": {"Y": -1}, "k": 0.01},
    ])


@pytest.mark.parametrize("mode,launch", [("FP64", {}), ("FP32", {}), ("MIX_F16_SR", {}), ("MIX_F16_RTN", {}),
                                         ("UNI_F16_SR", {}), ("UNI_BF16_SR_NORM", {}),
                                         ("MIX_F16_SR", {"block_size": 512}), ("FP64", {"block_size": 512})])
def test_zero_guards_at_low_counts(gpu, orc, mode, launch):
    # counts crossing the reactant orders: the guard-free and guarded
    # propensity versions must agree with the oracle's guarded definition
    run_both(gpu, orc, low_count_network(), np.array([0, 0], np.int32), 64 * 40, 20.0,
             wl.snapshot_grid(20.0, 21), mode, seed=5, **launch)


def largest_network():
    """32 species and 64 reactions (the C ABI's limits): per species a birth
    (every eighth one repressed by its neighbour through a Hill law) and a
    loss, the losses alternating between first order, a bimolecular reaction
    with the next species and a dimerisation. In the 16-bit modes its rounding
    fields outgrow the producer waves' LDS rings: mixed fp16 SR gets rings of
    depth 2, uniform fp16 SR none (the 512-thread kernel then runs eight
    event-loop waves that form their own draws)."""
    sp = [f"X{i}" for i in range(32)]
    rx = []
    for i in range(32):
        if i % 8 == 7:
            rx.append({"change": {sp[i]: +1}, "hill": ("repress", sp[i - 1], 0.5, 6.0, 4.0, 2)})
        else:
            rx.append({"change": {sp[i]: +1}, "k": 4.0 + (i % 3)})
        if i % 3 == 0:
            rx.append({"reactants": {sp[i]: 1}, "change": {sp[i]: -1}, "k": 0.6})
        elif i % 3 == 1:
            rx.append({"reactants": {sp[i]: 1, sp[(i + 1) % 32]: 1}, "change": {sp[i]: -1}, "k": 0.08})
        else:
            rx.append({"reactants": {sp[i]: 2}, "change": {sp[i]: -1}, "k": 0.05})
    return wl._build("largest", sp, rx)


@pytest.mark.parametrize("mode,launch", [("FP64", {}), ("MIX_F16_SR", {}), ("UNI_F16_SR", {}),
                                         ("FP64", {"block_size": 512}), ("MIX_F16_SR", {"block_size": 512}),
                                         ("UNI_F16_SR", {"block_size": 512}),
                                         # two producers for wave 0: with a ring of 16 slots (FP64),
                                         # and with one of 2 (mixed fp16 SR), where one producer stays
                                         ("FP64", {"block_size": 512, "placement": 197}),
                                         ("MIX_F16_SR", {"block_size": 512, "placement": 197})])
def test_largest_network(gpu, orc, mode, launch):
    m = largest_network()
    assert m.n_species == 32 and m.n_reactions == 64
    run_both(gpu, orc, m, np.full(32, 3, np.int32), 64 * 12, 2.0, wl.snapshot_grid(2.0, 5), mode, seed=9, **launch)


def run_records(gpu, orc, spec, x0, n, t_end, snap_t, mode, mask, cap, *, seed=1, **launch):
    m = gpu.Model(spec)
    item = {"model": m, "x0": x0, "n_traj": n, "record": (mask, cap)}
    print(f"[gpu-parity] records {spec.name} mode={mode} n={n} mask={mask} cap={cap} launch={launch}", flush=True)
    run = gpu.ssa_ensemble_run([item], t_end, snap_t, seed, mode, max_events=TEST_CAP, **launch)
    rec = run.records(0)
    ref = orc.simulate(spec, mode, x0, t_end, snap_t, seed, n_traj=n, record_mask=mask, record_cap=cap,
                       max_events=TEST_CAP, threads=ORACLE_THREADS)
    assert_parity(ref, run.snapshots(0), run.stats(0), mode, spec.name)
    np.testing.assert_array_equal(rec["n"], ref["rec_n"])
    for i in range(n):
        k = min(int(ref["rec_n"][i]), cap)
        np.testing.assert_array_equal(rec["j"][i, :k], ref["rec_j"][i, :k])
        np.testing.assert_array_equal(rec["t"][i, :k], ref["rec_t"][i, :k])
    return rec, ref


@pytest.mark.parametrize("mode", ["FP64", "FP32", "MIX_F16_SR", "UNI_BF16_SR_NORM"])
def test_event_record_matches_oracle(gpu, orc, mode):
    # gene switches of the telegraph model (reactions 0 and 1), as for the
    # dwell-time distributions; a capacity below some trajectories' counts
    spec = wl.telegraph(0.05, 0.05, 20.0, 1.0)
    x0 = np.array([1, 0, 0], np.int32)
    rec, ref = run_records(gpu, orc, spec, x0, 300, 200.0, wl.snapshot_grid(200.0, 11), mode, 0b11, 12, seed=4)
    assert (ref["rec_n"] > 12).any() and (ref["rec_n"] < 12).any()


def test_event_record_chunked_and_every_reaction(gpu, orc):
    # all reactions recorded (the log replays the trajectory) across snapshot
    # windows: the count is carried between launches
    spec = wl.telegraph(0.05, 0.05, 20.0, 1.0)
    x0 = np.array([1, 0, 0], np.int32)
    for chunks, window in ((1, 0), (3, 0), (2, 2)):
        run_records(gpu, orc, spec, x0, 130, 20.0, wl.snapshot_grid(20.0, 9), "MIX_F16_SR", 0b1111, 1200,
                    seed=2, n_chunks=chunks, first_window=window)


def test_event_record_in_a_batch(gpu, orc):
    # one item records, the other does not; both match the oracle
    tele, bd = wl.telegraph(0.05, 0.05, 20.0, 1.0), wl.birth_death(20.0, 1.0)
    items = [{"model": gpu.Model(tele), "x0": np.array([1, 0, 0], np.int32), "n_traj": 150, "record": (0b11, 20)},
             {"model": gpu.Model(bd), "x0": np.array([0], np.int32), "n_traj": 100}]
    print("[gpu-parity] records in a two-item batch", flush=True)
    run = gpu.ssa_ensemble_run(items, 50.0, [25.0, 50.0], 8, "FP64")
    ref = orc.simulate(tele, "FP64", items[0]["x0"], 50.0, [25.0, 50.0], 8, n_traj=150, record_mask=0b11,
                       record_cap=20, threads=ORACLE_THREADS)
    rec = run.records(0)
    np.testing.assert_array_equal(rec["n"], ref["rec_n"])
    k = np.minimum(ref["rec_n"], 20)
    for i in range(150):
        np.testing.assert_array_equal(rec["t"][i, :k[i]], ref["rec_t"][i, :k[i]])
    ref_bd = orc.simulate(bd, "FP64", items[1]["x0"], 50.0, [25.0, 50.0], 8, n_traj=100, traj_id_base=150,
                          threads=ORACLE_THREADS)
    np.testing.assert_array_equal(run.snapshots(1), ref_bd["snap"])
    with pytest.raises(gpu.SsaError):
        run.records(1)


def test_self_repressor_activation_and_repression(gpu, orc):
    spec = wl._build("hill_pair", ["X", "Y"], [
        {"change": {"X": +1}, "hill": ("repress", "Y", 1.0, 40.0, 15.0, 3)},
        {"reactants": {"X": 1}, "change": {"X": -1}, "k": 1.0},
        {"change": {"Y": +1}, "hill": ("activate", "X", 0.5, 30.0, 20.0, 2)},
        {"reactants": {"Y": 1}, "change": {"Y": -1}, "k": 0.7},
    ])
    for mode in ("FP64", "FP32", "MIX_BF16_SR", "UNI_F16_SR_NORM"):
        run_both(gpu, orc, spec, np.array([3, 0], np.int32), 700, 20.0, wl.snapshot_grid(20.0, 9), mode, seed=9)


@pytest.mark.parametrize("mode", ["MIX_F16_SR", "MIX_F16_RTN", "MIX_BF16_SR"])
def test_fp16_subnormal_propensities(gpu, orc, mode):
    """Rates around 1e-6 put every propensity in fp16's subnormal range, where
    stochastic rounding decides on fewer dropped-fraction bits."""
    m = wl.birth_death(3e-6, 2e-6)
    run_both(gpu, orc, m, np.array([3], np.int32), 3000, 4e5, [1e5, 2e5, 4e5], mode, seed=12)


def test_refill_path_single_workgroup(gpu, orc):
    """One workgroup of one wave runs 2,000 trajectories: every lane refills
    many times from the work counter."""
    W = wl.config_birth_death()
    it = W.items[0]
    run_both(gpu, orc, it.model, it.x0, 2000, 20.0, [5.0, 20.0], "MIX_F16_SR", seed=4,
             block_size=64, grid_size=1)


def test_ragged_and_tiny_ensembles(gpu, orc):
    W = wl.config_schlogl()
    it = W.items[0]
    for n in (1, 63, 65, 257):
        run_both(gpu, orc, it.model, it.x0, n, 1.0, wl.snapshot_grid(1.0, 5), "MIX_F16_SR", seed=5)


def test_chunked_graph_run_matches_single_launch(gpu, orc):
    W = wl.config_schlogl()
    it = W.items[0]
    for mode in ("FP64", "UNI_BF16_SR_NORM"):
        _, s1, st1 = run_both(gpu, orc, it.model, it.x0, 700, 5.0, wl.snapshot_grid(5.0, 51), mode, seed=6,
                              max_events=W.max_events)
        for chunks, reorder, window in ((4, 0, 0), (4, -1, 0), (2, 0, 5), (3, 0, 1), (3, -1, 49)):
            _, s4, st4 = run_both(gpu, orc, it.model, it.x0, 700, 5.0, wl.snapshot_grid(5.0, 51), mode, seed=6,
                                  max_events=W.max_events, n_chunks=chunks, reorder=reorder, first_window=window)
            np.testing.assert_array_equal(s1, s4)
            for k in st1:
                np.testing.assert_array_equal(st1[k], st4[k])


@pytest.mark.parametrize("mode,launch", [("FP64", {}), ("MIX_F16_SR", {}), ("FP64", {"block_size": 512}),
                                         ("MIX_F16_SR", {"block_size": 512})])
def test_graph_captured_chunks(gpu, orc, mode, launch):
    """More than 16 snapshot windows: the run's launches (the simulation
    kernel per window and the reorder kernels between windows) are captured
    into one hipGraph and launched as a graph. 25 windows over 51 rows, with
    a short first window and with even windows; results equal the single
    launch's and the oracle's."""
    W = wl.config_schlogl()
    it = W.items[0]
    ts = wl.snapshot_grid(5.0, 51)
    run1, s1, st1 = run_both(gpu, orc, it.model, it.x0, 900, 5.0, ts, mode, seed=6, max_events=W.max_events,
                             **launch)
    assert run1.info()["graph"] == 0
    for chunks, window, reorder in ((25, 0, 0), (25, 3, 0), (17, 0, -1), (50, 2, 0)):
        run, s, st = run_both(gpu, orc, it.model, it.x0, 900, 5.0, ts, mode, seed=6, max_events=W.max_events,
                              n_chunks=chunks, first_window=window, reorder=reorder, **launch)
        info = run.info()
        assert info["graph"] == 1 and info["n_launches"] == chunks, info
        np.testing.assert_array_equal(s1, s)
        for k in st1:
            np.testing.assert_array_equal(st1[k], st[k])


def test_special_statuses(gpu, orc):
    # absorbing: pure decay from 5
    run_both(gpu, orc, wl.birth_death(0.0, 1.0), np.array([5], np.int32), 300, 1e6, [0.0, 1e6], "FP64")
    # fp16 overflow at event 0 (zero-order constant 1e5 > 65504)
    _, s, st = run_both(gpu, orc, wl.birth_death(1e5, 1.0), np.array([250], np.int32), 130, 10.0,
                        [0.0, 5.0, 10.0], "MIX_F16_SR")
    assert np.all(st["status"] == 2) and np.all(s == 250)
    # event cap under uniform bf16 RTN
    _, _, st = run_both(gpu, orc, wl.birth_death(10.0, 0.1), np.array([0], np.int32), 200, 100.0,
                        [50.0, 100.0], "UNI_BF16_RTN", max_events=300)
    assert np.all(st["status"] == 3)


def test_no_snapshots_and_empty_item(gpu, orc):
    m = wl.birth_death()
    run_both(gpu, orc, m, np.array([0], np.int32), 100, 3.0, [], "FP64")
    mdl = gpu.Model(m)
    run = gpu.ssa_ensemble_run([{"model": mdl, "x0": [0], "n_traj": 0}], 3.0, [1.0], 1, "FP64")
    assert run.snapshots(0).shape == (1, 1, 0)


def test_multi_item_batch_matches_oracle_per_item(gpu, orc):
    """Five networks in one persistent launch; item m's trajectory ids start
    after the previous items' (traj_id_base + offset)."""
    W = wl.config_heterogeneous(n_traj_total=5 * 150)
    t_end, ts = 15.0, wl.snapshot_grid(15.0, 16)
    models = {}
    items = gpu.items_from_workload(W, models)
    for mode, chunks in (("FP64", 1), ("MIX_F16_SR", 1), ("MIX_BF16_SR", 1), ("MIX_F16_SR", 3)):
        print(f"[gpu-parity] heterogeneous mode={mode} chunks={chunks}", flush=True)
        run = gpu.ssa_ensemble_run(items, t_end, ts, 1, mode, traj_id_base=1000, max_events=W.max_events,
                                   n_chunks=chunks)
        base = 1000
        for i, it in enumerate(W.items):
            ref = orc.simulate(it.model, mode, it.x0, t_end, ts, 1, n_traj=it.n_traj, traj_id_base=base,
                               max_events=W.max_events, threads=ORACLE_THREADS)
            assert_parity(ref, run.snapshots(i), run.stats(i), mode, it.model.name)
            base += it.n_traj


def test_full_size_schlogl_sampled(gpu, orc):
    """The benchmark workload (100,000 trajectories) on a sample of trajectory
    ids spread over the whole range, in the default launch and in the
    benchmark's launch shapes: one event-loop wave per SIMD forming its own
    draws (1024 waves of 64) or paired with a draw-producing wave (256
    workgroups of 512), two snapshot windows with a first window of 10 or 15
    rows (the autotuner's choices for the two modes)."""
    W = wl.config_schlogl()
    it = W.items[0]
    sample = np.unique(np.concatenate([np.arange(0, 100_000, 997), [99_999, 65_535, 65_536]]))
    launches = ({}, dict(block_size=64, grid_size=1024, n_chunks=2, first_window=10),
                dict(block_size=512, grid_size=256, n_chunks=2, first_window=10),
                dict(block_size=512, grid_size=256, n_chunks=2, first_window=15))
    for mode in ("FP64", "MIX_F16_SR"):
        for launch in launches:
            run, snap, st = run_both(gpu, orc, it.model, it.x0, it.n_traj, W.t_end, W.snap_t, mode, seed=W.seed,
                                     max_events=W.max_events, indices=sample, **launch)
            assert np.all(run.stats(0)["status"] == 0)


def sampled_parity(gpu, orc, W, mode, samples, **launch):
    """Run workload W whole on the GPU and compare the trajectory ids in
    samples[i] (local to item i) with the oracle. Snapshot rows are gathered
    on the device, so the multi-gigabyte outputs never cross to the host."""
    import torch
    items = gpu.items_from_workload(W)
    print(f"[gpu-parity] full-size {W.name} mode={mode} n={W.n_traj} launch={launch}", flush=True)
    run = gpu.ssa_ensemble_run(items, W.t_end, W.snap_t, W.seed, mode, max_events=W.max_events, **launch)
    run.wait()
    base = 0
    for i, it in enumerate(W.items):
        idx = np.asarray(samples[i], dtype=np.int64)
        snap = run.tensors(i)[0][:, :, torch.from_numpy(idx).cuda()].cpu().numpy()
        st = {k: v[idx] for k, v in run.stats(i).items()}
        ref = orc.simulate(it.model, mode, it.x0, W.t_end, W.snap_t, W.seed, indices=idx, traj_id_base=base,
                           max_events=W.max_events, set_rate=it.set_rate, traj_per_set=it.traj_per_set,
                           threads=ORACLE_THREADS)
        assert_parity(ref, snap, st, mode, f"{W.name}/{it.model.name}")
        base += it.n_traj
    info = run.info()
    run.destroy()
    del run
    torch.cuda.empty_cache()
    return info


def spread(n, count, extra=()):
    """About `count` ids spread over range(n), plus its ends and `extra`."""
    ids = np.arange(0, n, max(1, n // count))
    return np.unique(np.concatenate([ids, [0, n - 1], np.asarray(extra, dtype=np.int64)]).astype(np.int64))


@pytest.mark.parametrize("mode", ["FP64", "UNI_F16_SR_NORM", "UNI_BF16_SR"])
def test_full_size_telegraph_sampled(gpu, orc, mode):
    """Telegraph, 1,000,000 trajectories to T_end = 200 with 201 snapshot
    rows (2.4 GB of snapshots), in the default launch."""
    W = wl.config_telegraph()
    sampled_parity(gpu, orc, W, mode, [spread(W.n_traj, 120, [65_535, 65_536, 524_287])])


# the launches the benchmark's autotuner chooses for the sweep (256 workgroups of
# 512 threads, two windows, the first of 7 rows): MIX_F16_SR with wave 0 fed by two
# producers (197), FP64 with wave 0 alone and fed first (29)
BENCH_DIMER = {"MIX_F16_SR": dict(block_size=512, grid_size=256, n_chunks=2, first_window=7, placement=197),
               "FP64": dict(block_size=512, grid_size=256, n_chunks=2, first_window=7, placement=29)}


@pytest.mark.parametrize("launch", ["default", "bench"])
@pytest.mark.parametrize("mode", ["FP64", "MIX_F16_SR"])
def test_full_size_dimer_sweep_sampled(gpu, orc, mode, launch):
    """Open dimer, 4,096 parameter sets x 256 trajectories in one launch,
    lengths spread over three decades: ids spread over the sets plus both ends
    of the sets with the largest and smallest production rate; in the default
    launch and in the one the benchmark times."""
    W = wl.config_dimer_sweep()
    it = W.items[0]
    hi, lo = int(np.argmax(it.set_rate[:, 0])), int(np.argmin(it.set_rate[:, 0]))
    tps = it.traj_per_set
    extra = [hi * tps, hi * tps + tps - 1, lo * tps, lo * tps + tps - 1]
    kw = BENCH_DIMER[mode] if launch == "bench" else {}
    info = sampled_parity(gpu, orc, W, mode, [spread(W.n_traj, 100, extra)], **kw)
    if kw:
        assert info["placement"] == kw["placement"] | 1


@pytest.mark.parametrize("mode,launch", [("FP64", {}), ("MIX_F16_SR", dict(block_size=512, grid_size=256)),
                                         ("MIX_BF16_SR", dict(block_size=512, grid_size=256))])
def test_full_size_heterogeneous_sampled(gpu, orc, mode, launch):
    """All five networks in one launch, 800,000 trajectories each, to
    T_end = 500 with 501 snapshot rows (20.8 GB of snapshots; item ids and
    snapshot offsets beyond 2^31 elements): 16 ids per network."""
    W = wl.config_heterogeneous()
    info = sampled_parity(gpu, orc, W, mode, [spread(it.n_traj, 14) for it in W.items], **launch)
    assert info["total_events"] > 10 ** 12


# ---------------------------------------------------------------------------
# Producer waves (block_size 512): waves 0-3 of a workgroup run trajectories,
# wave w + 4 forms wave w's draws ahead through an LDS ring. Same results as
# every other launch shape, so the same oracle bar.
# ---------------------------------------------------------------------------
PC = dict(block_size=512)


@pytest.mark.parametrize("mode", ["FP64", "FP32", "MIX_F16_SR", "MIX_BF16_SR", "UNI_BF16_SR_NORM", "UNI_F16_SRA"])
def test_producer_waves_schlogl(gpu, orc, mode):
    W = wl.config_schlogl()
    it = W.items[0]
    run_both(gpu, orc, it.model, it.x0, 1500, W.t_end, W.snap_t, mode, seed=W.seed, max_events=W.max_events, **PC)


def test_producer_waves_one_workgroup_refills(gpu, orc):
    """One workgroup: four event-loop waves and their producers run 3,000
    trajectories, so every lane claims many trajectories, each a new epoch of
    its ring slots."""
    W = wl.config_birth_death()
    it = W.items[0]
    for mode in ("MIX_F16_SR", "FP64", "UNI_F16_SR_NORM"):
        run_both(gpu, orc, it.model, it.x0, 3000, 20.0, [5.0, 20.0], mode, seed=4, block_size=512, grid_size=1)


@pytest.mark.parametrize("mode", ["MIX_F16_SR", "UNI_BF16_SRA"])
def test_producer_waves_hill_laws(gpu, orc, mode):
    m = wl.repressilator()
    run_both(gpu, orc, m, np.array([0, 0, 0, 0, 0, 20], np.int32), 600, 60.0, wl.snapshot_grid(60.0, 61),
             mode, seed=3, max_events=10_000_000, **PC)


def test_producer_waves_count_conversion(gpu, orc):
    levels, kd = (1500.0, 2100.0, 2600.0), 1.0
    rates = np.array([[kb, kd] for kb in levels], np.float64)
    run_both(gpu, orc, wl.birth_death(levels[1], kd), np.array([2100], np.int32), 3 * 70, 1.5,
             wl.snapshot_grid(1.5, 7), "MIX_F16_SR", seed=11, set_rate=rates, traj_per_set=70,
             max_events=200_000, **PC)


def test_producer_waves_chunked_and_suspended(gpu, orc):
    W = wl.config_schlogl()
    it = W.items[0]
    for mode in ("MIX_F16_SR", "UNI_BF16_SR_NORM"):
        for chunks, window in ((3, 0), (2, 5)):
            run_both(gpu, orc, it.model, it.x0, 700, 5.0, wl.snapshot_grid(5.0, 51), mode, seed=6,
                     max_events=W.max_events, n_chunks=chunks, first_window=window, **PC)


def test_producer_waves_multi_item_batch(gpu, orc):
    """Five networks in one launch: each event-loop wave hands its producer
    from one item (and draw layout) to the next."""
    W = wl.config_heterogeneous(n_traj_total=5 * 150)
    t_end, ts = 15.0, wl.snapshot_grid(15.0, 16)
    items = gpu.items_from_workload(W, {})
    for mode, chunks, grid in (("FP64", 1, 0), ("MIX_F16_SR", 1, 1), ("UNI_F16_SR_NORM", 3, 0)):
        print(f"[gpu-parity] producer waves, heterogeneous mode={mode} chunks={chunks} grid={grid}", flush=True)
        run = gpu.ssa_ensemble_run(items, t_end, ts, 1, mode, traj_id_base=1000, max_events=W.max_events,
                                   n_chunks=chunks, block_size=512, grid_size=grid)
        base = 1000
        for i, it in enumerate(W.items):
            ref = orc.simulate(it.model, mode, it.x0, t_end, ts, 1, n_traj=it.n_traj, traj_id_base=base,
                               max_events=W.max_events, threads=ORACLE_THREADS)
            assert_parity(ref, run.snapshots(i), run.stats(i), mode, it.model.name)
            base += it.n_traj


def test_producer_waves_event_record(gpu, orc):
    spec = wl.telegraph(0.05, 0.05, 20.0, 1.0)
    x0 = np.array([1, 0, 0], np.int32)
    run_records(gpu, orc, spec, x0, 300, 200.0, wl.snapshot_grid(200.0, 11), "MIX_F16_SR", 0b11, 12, seed=4, **PC)


# ---------------------------------------------------------------------------
# Placements of the 512-thread launch (producer on the event-loop wave's own
# SIMD or the next one, wave-major first claims, wave 0 alone on its SIMD,
# wave priorities, three event-loop waves with wave 0's producer alone on a
# SIMD, two producers splitting wave 0's draws by event parity): only where and
# when work runs changes, so results are the oracle's in every one.
# ---------------------------------------------------------------------------
PLACEMENTS = [3, 5, 7, 9, 13, 29, 45, 19, 35, 65, 69, 85, 101, 197, 213]


@pytest.mark.parametrize("placement", PLACEMENTS)
@pytest.mark.parametrize("mode", ["FP64", "MIX_F16_SR"])
def test_placements_schlogl(gpu, orc, mode, placement):
    W = wl.config_schlogl()
    it = W.items[0]
    run, _, _ = run_both(gpu, orc, it.model, it.x0, 1500, W.t_end, W.snap_t, mode, seed=W.seed,
                         max_events=W.max_events, block_size=512, grid_size=2, n_chunks=2, first_window=10,
                         placement=placement)
    assert run.info()["placement"] == placement


@pytest.mark.parametrize("placement", [1, 7, 13, 29, 45, 69, 197, 213])
def test_placements_dimer_sets_with_conversion_fields(gpu, orc, placement):
    """Per-lane parameter sets whose counts pass the fp16 exact-integer limit
    (2048): the producers form the conversion fields for those lanes, under
    every placement."""
    rates = np.array([[400.0, 0.1, 0.001, 0.5], [50.0, 0.1, 0.001, 0.5], [900.0, 0.3, 0.0005, 0.5]], np.float64)
    m = wl.dimer_open()
    run, snap, _ = run_both(gpu, orc, m, np.array([3000, 8000], np.int32), 3 * 100, 1.5,
                            wl.snapshot_grid(1.5, 4), "MIX_F16_SR", seed=31, set_rate=rates, traj_per_set=100,
                            max_events=3_000_000, block_size=512, grid_size=1, n_chunks=2, first_window=1,
                            placement=placement)
    assert snap[:, 0, :].max() > 2048
