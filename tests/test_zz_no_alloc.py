"""ssa_ensemble_run_noalloc (the allocation-free variant of ssa_ensemble_run)
against ssa_ensemble_run on the same inputs, through the C ABI: snapshots,
event counts, statuses and last-event times bit-identical, on two calls in a
row (the second with a smaller ensemble, so stale counters, carry state or
claim order in the shared scratch array would show), in a chunked launch with
producer waves and a single launch; plus its refusals."""
import numpy as np
import pytest

from paper_2605_00479_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    from paper_2605_00479_amd import ssa
    ssa.lib()
    return ssa


def outputs_for(n_species, n_traj, n_snap):
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    return [(torch.full((n_snap, n_species, n_traj), -7, dtype=torch.int32, device=dev),
             torch.full((n_traj,), -7, dtype=torch.int64, device=dev),
             torch.full((n_traj,), -7.0, dtype=torch.float64, device=dev),
             torch.full((n_traj,), 77, dtype=torch.uint8, device=dev))]


def compare(gpu, items, t_end, ts, seed, mode, cap, **launch):
    import torch
    print(f"[no-alloc] {mode} n={items[0]['n_traj']} seed={seed} launch={launch}", flush=True)
    ref = gpu.ssa_ensemble_run(items, t_end, ts, seed, mode, max_events=cap, **launch)
    ref_snap, ref_st = ref.snapshots(0), ref.stats(0)
    out = outputs_for(items[0]["model"].n_species, items[0]["n_traj"], len(ts))
    gpu.ssa_ensemble_run_noalloc(items, t_end, ts, seed, mode, out, max_events=cap, **launch)
    torch.cuda.current_stream().synchronize()
    snap, nev, tl, st = (t.cpu().numpy() for t in out[0])
    np.testing.assert_array_equal(snap, ref_snap)
    np.testing.assert_array_equal(nev.astype(np.uint64), ref_st["n_events"])
    np.testing.assert_array_equal(tl, ref_st["t_last"])
    np.testing.assert_array_equal(st, ref_st["status"])
    return ref_st


@pytest.mark.parametrize("mode,launch", [
    ("MIX_F16_SR", dict(block_size=512, grid_size=8, n_chunks=3, first_window=5)),
    ("FP64", dict(block_size=256, grid_size=4, n_chunks=1)),
    ("UNI_BF16_SR_NORM", dict(block_size=64, grid_size=16, n_chunks=4)),
])
def test_noalloc_matches_ensemble_run_twice(gpu, mode, launch):
    W = wl.config_schlogl()
    it = W.items[0]
    model = gpu.Model(it.model)
    ts = wl.snapshot_grid(5.0, 51)
    big = [{"model": model, "x0": it.x0, "n_traj": 3000}]
    small = [{"model": model, "x0": it.x0, "n_traj": 700}]
    st = compare(gpu, big, 5.0, ts, 6, mode, W.max_events, **launch)
    assert st["n_events"].sum() > 0
    compare(gpu, small, 5.0, ts, 9, mode, W.max_events, **launch)


def test_noalloc_refusals(gpu):
    import torch
    W = wl.config_schlogl()
    it = W.items[0]
    model = gpu.Model(it.model)
    ts = wl.snapshot_grid(5.0, 51)
    items = [{"model": model, "x0": it.x0, "n_traj": 100}]
    gpu.ssa_ensemble_run(items, 5.0, ts, 1, "MIX_F16_RTN", max_events=W.max_events).wait()
    # outputs missing
    with pytest.raises(gpu.SsaError) as e:
        out = outputs_for(1, 100, len(ts))
        gpu.ssa_ensemble_run_noalloc(items, 5.0, ts, 1, "MIX_F16_RTN",
                                     [(out[0][0], torch.empty(0), out[0][2], out[0][3])], max_events=W.max_events)
    assert e.value.code == gpu.SSA_E_INVALID
    # a network whose kernel no run has loaded yet
    other = [{"model": gpu.Model(wl.birth_death(3.0, 0.25)), "x0": [0], "n_traj": 100}]
    with pytest.raises(gpu.SsaError) as e:
        gpu.ssa_ensemble_run_noalloc(other, 5.0, ts, 1, "MIX_BF16_RTN", outputs_for(1, 100, len(ts)),
                                     max_events=W.max_events)
    assert e.value.code == gpu.SSA_E_INVALID and "not loaded" in str(e.value)
    # a chunked run whose carry state outgrows the scratch array
    n = 3_000_000
    with pytest.raises(gpu.SsaError) as e:
        gpu.ssa_ensemble_run_noalloc([{"model": model, "x0": it.x0, "n_traj": n}], 5.0, [2.5, 5.0], 1,
                                     "MIX_F16_RTN", outputs_for(1, n, 2), max_events=W.max_events, n_chunks=2)
    assert e.value.code == gpu.SSA_E_INVALID and "scratch" in str(e.value)
    # the array is still usable afterwards
    compare(gpu, items, 5.0, ts, 1, "MIX_F16_RTN", W.max_events, n_chunks=2, block_size=256, grid_size=2)
