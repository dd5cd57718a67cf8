"""C ABI checks that need no GPU: the library loads, exports every function
include/ssa_rp.h declares, validates arguments with the documented codes,
and compiles kernels for every precision mode (hipRTC, gfx950)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2605_00479_amd import ssa, workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ssa_rp.h")).read()
    return sorted(set(re.findall(r"^(?:int|void|const char \*)\s*\*?\s*(ssa_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = ssa.lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert ssa.lib().ssa_version().startswith(b"ssa_rp")


def test_binding_names_match_the_abi():
    assert set(ssa.EXPORTS) == set(declared_functions())


def _law(kind=0, k=1.0, reg=0, h=1, basal=0.0, K=1.0):
    return ssa.ssa_law(kind, reg, h, 0, k, basal, K)


def _create(N, M, order, nu, laws):
    h = ctypes.c_void_p()
    o = np.ascontiguousarray(order, np.int32)
    n = np.ascontiguousarray(nu, np.int32)
    arr = (ssa.ssa_law * len(laws))(*laws)
    rc = ssa.lib().ssa_model_create(N, M, o.ctypes.data if o.size else None, n.ctypes.data if n.size else None,
                                    ctypes.addressof(arr), ctypes.byref(h))
    if rc == 0:
        ssa.lib().ssa_model_destroy(h)
    return rc


def test_model_create_validation():
    ok = _create(1, 2, [[0], [1]], [[1], [-1]], [_law(k=10.0), _law(k=0.1)])
    assert ok == ssa.SSA_OK
    assert _create(0, 1, [[0]], [[1]], [_law()]) == ssa.SSA_E_INVALID
    assert _create(1, 1, [[-1]], [[1]], [_law()]) == ssa.SSA_E_INVALID
    assert _create(1, 1, [[0]], [[1]], [_law(k=-1.0)]) == ssa.SSA_E_INVALID
    assert _create(1, 1, [[0]], [[1]], [_law(k=float("nan"))]) == ssa.SSA_E_INVALID
    assert _create(1, 1, [[5]], [[1]], [_law()]) == ssa.SSA_E_UNSUPPORTED
    assert _create(1, 1, [[0]], [[1]], [_law(kind=1, reg=1)]) == ssa.SSA_E_INVALID
    assert _create(1, 1, [[0]], [[1]], [_law(kind=1, h=0)]) == ssa.SSA_E_INVALID
    assert _create(1, 1, [[0]], [[1]], [_law(kind=1, K=0.0)]) == ssa.SSA_E_INVALID
    assert _create(1, 1, [[0]], [[5000]], [_law()]) == ssa.SSA_E_INVALID
    assert _create(1, 1, [[0]], [[1]], [_law(kind=7)]) == ssa.SSA_E_INVALID
    assert ssa.lib().ssa_last_error() != b""


def _run_rc(**over):
    m = ssa.Model(wl.birth_death())
    items = [{"model": m, "x0": [0], "n_traj": 10}]
    kw = dict(t_end=1.0, snap_t=[0.5, 1.0], seed=1, mode="FP64")
    kw.update(over)
    mode = kw.pop("mode")
    d, keep = ssa._desc(items, kw["t_end"], kw["snap_t"], kw["seed"], mode)
    for k, v in over.get("_fields", {}).items():
        setattr(d, k, v)
    return ssa.lib().ssa_prepare(ctypes.byref(d))


def test_run_descriptor_validation():
    assert _run_rc() == ssa.SSA_OK
    assert _run_rc(t_end=0.0) == ssa.SSA_E_INVALID
    assert _run_rc(t_end=float("inf")) == ssa.SSA_E_INVALID
    assert _run_rc(snap_t=[1.0, 0.5]) == ssa.SSA_E_INVALID
    assert _run_rc(snap_t=[2.0]) == ssa.SSA_E_INVALID
    assert _run_rc(_fields={"format": 9}) == ssa.SSA_E_INVALID
    assert _run_rc(_fields={"accum": 1}) == ssa.SSA_E_INVALID            # FP64 + uniform
    assert _run_rc(mode="MIX_F16_SR", _fields={"norm": 1}) == ssa.SSA_E_UNSUPPORTED
    assert _run_rc(mode="MIX_F16_SR", _fields={"rounding": 2}) == ssa.SSA_E_UNSUPPORTED
    assert _run_rc(mode="UNI_F16_SR", _fields={"rounding": 3}) == ssa.SSA_E_INVALID
    assert _run_rc(_fields={"block_size": 100}) == ssa.SSA_E_INVALID
    assert _run_rc(_fields={"block_size": 320}) == ssa.SSA_E_INVALID    # above 256, and not the paired 512
    assert _run_rc(_fields={"block_size": 1024}) == ssa.SSA_E_INVALID
    assert _run_rc(_fields={"n_items": 0}) == ssa.SSA_E_INVALID
    assert _run_rc(_fields={"traj_id_base": 2**32 - 5}) == ssa.SSA_E_INVALID
    assert _run_rc(_fields={"reorder": 2}) == ssa.SSA_E_INVALID
    assert _run_rc(_fields={"first_window": -1}) == ssa.SSA_E_INVALID
    # two snapshot rows cannot hold a first window of 2 and one more window
    assert _run_rc(_fields={"n_chunks": 2, "first_window": 2}) == ssa.SSA_E_INVALID
    assert _run_rc(_fields={"n_chunks": 2, "first_window": 1}) == ssa.SSA_OK
    # placement: 0, or SSA_PLACE_EXPLICIT with known flags
    every_flag = (ssa.PLACE_EXPLICIT | ssa.PLACE_NEIGHBOUR_PRODUCER | ssa.PLACE_WAVE_MAJOR | ssa.PLACE_SOLO_WAVE0 |
                  ssa.PLACE_FEED_WAVE0 | ssa.PLACE_PRODUCER_FIRST | ssa.PLACE_DEDICATED_FEED0 | ssa.PLACE_TWO_FEED0)
    assert _run_rc(_fields={"placement": every_flag}) == ssa.SSA_OK
    assert _run_rc(_fields={"placement": ssa.PLACE_FEED_WAVE0}) == ssa.SSA_E_INVALID      # no SSA_PLACE_EXPLICIT
    assert _run_rc(_fields={"placement": every_flag | 256}) == ssa.SSA_E_INVALID         # unknown flag
    # two producers for wave 0: only with the dedicated placement
    assert _run_rc(_fields={"placement": ssa.PLACE_EXPLICIT | ssa.PLACE_TWO_FEED0}) == ssa.SSA_E_INVALID
    # wave 0 alone on its SIMD: one-item launches only
    m2 = ssa.Model(wl.birth_death())
    two = [{"model": m2, "x0": [0], "n_traj": 10}, {"model": m2, "x0": [1], "n_traj": 10}]
    d2, keep2 = ssa._desc(two, 1.0, [0.5, 1.0], 1, "FP64")
    d2.placement = ssa.PLACE_EXPLICIT | ssa.PLACE_SOLO_WAVE0
    assert ssa.lib().ssa_prepare(ctypes.byref(d2)) == ssa.SSA_E_INVALID
    d2.placement = ssa.PLACE_EXPLICIT | ssa.PLACE_DEDICATED_FEED0
    assert ssa.lib().ssa_prepare(ctypes.byref(d2)) == ssa.SSA_OK
    d2.placement = ssa.PLACE_EXPLICIT | ssa.PLACE_DEDICATED_FEED0 | ssa.PLACE_TWO_FEED0
    assert ssa.lib().ssa_prepare(ctypes.byref(d2)) == ssa.SSA_E_INVALID
    with pytest.raises(ValueError):
        ssa.parse_mode("MIX_F8_SR")


def test_record_arguments_validated():
    m = ssa.Model(wl.telegraph(0.05, 0.05, 20.0, 1.0))

    def rc(mask, cap, n=10):
        d, keep = ssa._desc([{"model": m, "x0": [1, 0, 0], "n_traj": n, "record": (mask, cap)}], 1.0, [1.0], 1,
                            "FP64")
        return ssa.lib().ssa_prepare(ctypes.byref(d))

    assert rc(0b11, 16) == ssa.SSA_OK
    assert rc(0, 0) == ssa.SSA_OK
    assert rc(0b11, -1) == ssa.SSA_E_INVALID
    assert rc(0b11, (1 << 20) + 1) == ssa.SSA_E_INVALID
    assert rc(0b11, 1 << 20, n=4096) == ssa.SSA_E_INVALID       # cap * n_traj > 2^31
    assert rc(1 << 4, 16) == ssa.SSA_E_INVALID                    # the telegraph has 4 reactions


def test_negative_initial_count_rejected():
    m = ssa.Model(wl.birth_death())
    d, keep = ssa._desc([{"model": m, "x0": [-1], "n_traj": 4}], 1.0, [1.0], 1, "FP64")
    assert ssa.lib().ssa_prepare(ctypes.byref(d)) == ssa.SSA_E_INVALID


@pytest.mark.parametrize("mode", ["FP64", "FP32", "MIX_F16_RTN", "MIX_F16_SR", "MIX_BF16_RTN", "MIX_BF16_SR",
                                  "UNI_F16_RTN", "UNI_F16_SR", "UNI_F16_SR_NORM", "UNI_BF16_RTN",
                                  "UNI_BF16_SR", "UNI_BF16_SR_NORM", "UNI_F16_SRA", "UNI_BF16_SRA_NORM"])
def test_kernels_compile_for_every_mode(mode):
    W = wl.config_heterogeneous(100)
    items = ssa.items_from_workload(W)
    ssa.ssa_prepare(items, W.t_end, W.snap_t, mode, max_events=W.max_events)


@pytest.mark.parametrize("mode", ["FP32", "MIX_F16_SR", "MIX_BF16_RTN", "UNI_BF16_RTN", "UNI_F16_SR_NORM"])
def test_clocks_that_can_stall_need_an_event_cap(mode):
    """A binary32 or 16-bit clock stops advancing once the waiting time is
    below half its spacing: a run in such a mode must name a finite cap. The
    run is refused before anything reaches a GPU (ssa_ensemble_run validates
    first), so this needs none."""
    m = ssa.Model(wl.birth_death())
    items = [{"model": m, "x0": [0], "n_traj": 10}]
    for fn in ("ssa_prepare", "ssa_ensemble_run"):
        d, keep = ssa._desc(items, 1.0, [1.0], 1, mode, max_events=0)
        args = [ctypes.byref(d)] + ([ctypes.byref(ctypes.c_void_p())] if fn == "ssa_ensemble_run" else [])
        assert getattr(ssa.lib(), fn)(*args) == ssa.SSA_E_INVALID, fn
        assert b"max_events" in ssa.lib().ssa_last_error()
    d, keep = ssa._desc(items, 1.0, [1.0], 1, mode, max_events=1000)
    assert ssa.lib().ssa_prepare(ctypes.byref(d)) == ssa.SSA_OK
    d, keep = ssa._desc(items, 1.0, [1.0], 1, "FP64", max_events=0)
    assert ssa.lib().ssa_prepare(ctypes.byref(d)) == ssa.SSA_OK
