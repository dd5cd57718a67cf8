"""Thin ctypes binding of libssa_rp.so (the C ABI in include/ssa_rp.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels the library compiles. PyTorch provides device memory for the outputs
and the stream the run is queued on. The binding refuses to run if the
library is not built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssa_rp.so")

SSA_OK, SSA_E_INVALID, SSA_E_NOMEM, SSA_E_DEVICE, SSA_E_UNSUPPORTED, SSA_E_COMPILE = range(6)
FMT = {"FP64": 0, "FP32": 1, "F16": 2, "BF16": 3}
STATUS_NAMES = ("DONE", "ABSORBED", "OVERFLOW", "CAPPED")


class SsaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ssa error {code}: {msg}")
        self.code = code


class ssa_law(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("regulator", ctypes.c_int32), ("h", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("k", ctypes.c_double), ("basal", ctypes.c_double),
                ("K", ctypes.c_double)]


class ssa_item(ctypes.Structure):
    _fields_ = [("model", ctypes.c_void_p), ("x0", ctypes.c_void_p), ("n_traj", ctypes.c_int64),
                ("set_rates", ctypes.c_void_p), ("n_sets", ctypes.c_int64), ("traj_per_set", ctypes.c_int64),
                ("d_snap", ctypes.c_void_p), ("d_n_events", ctypes.c_void_p), ("d_t_last", ctypes.c_void_p),
                ("d_status", ctypes.c_void_p), ("record_mask", ctypes.c_uint64), ("record_cap", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("d_rec_t", ctypes.c_void_p), ("d_rec_j", ctypes.c_void_p),
                ("d_rec_n", ctypes.c_void_p)]


class ssa_run_desc(ctypes.Structure):
    _fields_ = [("items", ctypes.c_void_p), ("n_items", ctypes.c_int32), ("n_snap", ctypes.c_int32),
                ("t_end", ctypes.c_double), ("snap_t", ctypes.c_void_p), ("seed", ctypes.c_uint64),
                ("traj_id_base", ctypes.c_uint32), ("format", ctypes.c_int32), ("accum", ctypes.c_int32),
                ("rounding", ctypes.c_int32), ("norm", ctypes.c_int32), ("n_chunks", ctypes.c_int32),
                ("max_events", ctypes.c_uint64), ("hip_stream", ctypes.c_void_p),
                ("block_size", ctypes.c_int32), ("grid_size", ctypes.c_int32), ("reorder", ctypes.c_int32),
                ("first_window", ctypes.c_int32), ("placement", ctypes.c_int32)]


class ssa_run_info(ctypes.Structure):
    _fields_ = [("elapsed_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("n_launches", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("grid_size", ctypes.c_int32), ("vgprs", ctypes.c_int32),
                ("total_events", ctypes.c_uint64), ("first_window", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("placement", ctypes.c_int32)]


class ssa_tune_result(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_int32), ("grid_size", ctypes.c_int32), ("n_chunks", ctypes.c_int32),
                ("first_window", ctypes.c_int32), ("placement", ctypes.c_int32), ("n_candidates", ctypes.c_int32),
                ("best_ms", ctypes.c_double)]


EXPORTS = ("ssa_autotune", "ssa_model_create", "ssa_model_destroy", "ssa_ensemble_run", "ssa_run_wait",
           "ssa_snapshots_get", "ssa_run_stats_get", "ssa_run_info_get", "ssa_run_destroy",
           "ssa_last_error", "ssa_version", "ssa_prepare", "ssa_dump_source", "ssa_kernel_file",
           "ssa_records_get", "ssa_ensemble_run_noalloc")

_lib = None


def lib():
    """Load libssa_rp.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2605_00479_amd.csrc.build`")
        # torch ships its own HIP runtime under the same soname; loading torch first makes
        # this library bind to that one, so the process holds a single HIP runtime.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        L.ssa_model_create.argtypes = [i32, i32, vp, vp, vp, ctypes.POINTER(vp)]
        L.ssa_model_destroy.argtypes = [vp]
        L.ssa_model_destroy.restype = None
        L.ssa_ensemble_run.argtypes = [ctypes.POINTER(ssa_run_desc), ctypes.POINTER(vp)]
        L.ssa_run_wait.argtypes = [vp]
        L.ssa_snapshots_get.argtypes = [vp, i32, vp, ctypes.c_size_t, ctypes.c_int]
        L.ssa_run_stats_get.argtypes = [vp, i32, vp, vp, vp, ctypes.c_int]
        L.ssa_records_get.argtypes = [vp, i32, vp, vp, vp, ctypes.c_int]
        L.ssa_run_info_get.argtypes = [vp, ctypes.POINTER(ssa_run_info)]
        L.ssa_run_destroy.argtypes = [vp]
        L.ssa_run_destroy.restype = None
        L.ssa_last_error.restype = ctypes.c_char_p
        L.ssa_version.restype = ctypes.c_char_p
        L.ssa_prepare.argtypes = [ctypes.POINTER(ssa_run_desc)]
        L.ssa_dump_source.argtypes = [ctypes.POINTER(ssa_run_desc), ctypes.c_char_p]
        L.ssa_kernel_file.argtypes = [ctypes.POINTER(ssa_run_desc), ctypes.c_char_p, ctypes.c_size_t]
        L.ssa_autotune.argtypes = [ctypes.POINTER(ssa_run_desc), ctypes.POINTER(ssa_tune_result)]
        L.ssa_ensemble_run_noalloc.argtypes = [ctypes.POINTER(ssa_run_desc)]
        _lib = L
    return _lib


def _check(rc):
    if rc != SSA_OK:
        raise SsaError(rc, lib().ssa_last_error().decode())


def parse_mode(name: str):
    """FP64 / FP32 / {MIX,UNI}_{F16,BF16}_{RTN,SR,SRA}[_NORM] -> (format, accum, rounding, norm).
    SRA: stochastic rounding at accumulation points only (uniform mode)."""
    if name in ("FP64", "FP32"):
        return FMT[name], 0, 0, 0
    parts = name.split("_")
    if len(parts) not in (3, 4) or parts[0] not in ("MIX", "UNI") or parts[1] not in ("F16", "BF16") \
            or parts[2] not in ("RTN", "SR", "SRA") or (len(parts) == 4 and parts[3] != "NORM"):
        raise ValueError(f"unknown precision mode {name!r}")
    return FMT[parts[1]], int(parts[0] == "UNI"), {"RTN": 0, "SR": 1, "SRA": 2}[parts[2]], int(len(parts) == 4)


class Model:
    """An ssa_model handle built from a workloads.ModelSpec-like object."""

    def __init__(self, spec):
        N, M = int(spec.n_species), int(spec.n_reactions)
        order = np.ascontiguousarray(spec.order, dtype=np.int32).reshape(M, N)
        nu = np.ascontiguousarray(spec.nu, dtype=np.int32).reshape(M, N)
        laws = (ssa_law * M)()
        for j in range(M):
            laws[j].kind = int(spec.law[j])
            laws[j].k = float(spec.rate[j])
            laws[j].regulator = int(spec.hill_reg[j])
            laws[j].h = int(spec.hill_h[j])
            laws[j].basal = float(spec.hill_b[j])
            laws[j].K = float(spec.hill_K[j])
        h = ctypes.c_void_p()
        _check(lib().ssa_model_create(N, M, order.ctypes.data, nu.ctypes.data, ctypes.addressof(laws),
                                      ctypes.byref(h)))
        self.handle = h
        self.n_species, self.n_reactions = N, M

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ssa_model_destroy(self.handle)
            self.handle = None


class Run:
    """A queued ensemble run; results are read through the C ABI getters."""

    def __init__(self, handle, items, keep, record_caps=None):
        self.handle = handle
        self.items = items     # list of (N, E, K)
        self._keep = keep      # host arrays and output tensors referenced by the run
        self.record_caps = record_caps or [0] * len(items)

    def wait(self):
        _check(lib().ssa_run_wait(self.handle))

    def snapshots(self, item: int = 0) -> np.ndarray:
        N, E, K = self.items[item]
        out = np.empty((K, N, E), dtype=np.int32)
        _check(lib().ssa_snapshots_get(self.handle, item, out.ctypes.data, out.size, 0))
        return out

    def stats(self, item: int = 0) -> dict:
        N, E, K = self.items[item]
        nev = np.empty(E, dtype=np.uint64)
        tl = np.empty(E, dtype=np.float64)
        st = np.empty(E, dtype=np.uint8)
        _check(lib().ssa_run_stats_get(self.handle, item, nev.ctypes.data, tl.ctypes.data, st.ctypes.data, 0))
        return {"n_events": nev, "t_last": tl, "status": st}

    def records(self, item: int = 0) -> dict:
        """The item's event record: ``t`` [E, cap] float64 (clock after each
        recorded firing), ``j`` [E, cap] uint8 (reaction) and ``n`` [E]
        uint32 (recorded firings, also those past cap)."""
        N, E, K = self.items[item]
        cap = self.record_caps[item]
        t = np.empty((E, cap), dtype=np.float64)
        j = np.empty((E, cap), dtype=np.uint8)
        n = np.empty(E, dtype=np.uint32)
        _check(lib().ssa_records_get(self.handle, item, t.ctypes.data, j.ctypes.data, n.ctypes.data, 0))
        return {"t": t, "j": j, "n": n}

    def info(self) -> dict:
        inf = ssa_run_info()
        _check(lib().ssa_run_info_get(self.handle, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in ssa_run_info._fields_}

    def tensors(self, item: int = 0):
        """The caller-owned device output tensors of an item (snap, n_events, t_last, status)."""
        return self._keep["out"][item]

    def destroy(self):
        if self.handle:
            lib().ssa_run_destroy(self.handle)
            self.handle = None

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ssa_run_destroy(self.handle)
            self.handle = None


def _desc(items, t_end, snap_t, seed, mode, *, max_events=0, traj_id_base=0, n_chunks=1,
          block_size=0, grid_size=0, reorder=0, first_window=0, placement=0, stream=None, outputs=None):
    """Build an ssa_run_desc. items: list of dicts with model (Model), x0, n_traj,
    optional set_rates [n_sets, M] and traj_per_set, optional record =
    (reaction mask, records per trajectory)."""
    keep = {"arrays": [], "out": []}
    arr = (ssa_item * len(items))()
    for i, it in enumerate(items):
        m = it["model"]
        x0 = np.ascontiguousarray(it["x0"], dtype=np.int32)
        keep["arrays"].append(x0)
        arr[i].model = m.handle
        arr[i].x0 = x0.ctypes.data
        arr[i].n_traj = int(it["n_traj"])
        sr = it.get("set_rates")
        if sr is not None:
            sr = np.ascontiguousarray(sr, dtype=np.float64)
            keep["arrays"].append(sr)
            arr[i].set_rates = sr.ctypes.data
            arr[i].n_sets = sr.shape[0]
            arr[i].traj_per_set = int(it["traj_per_set"])
        rec = it.get("record")
        if rec is not None:
            arr[i].record_mask = int(rec[0]) & (2**64 - 1)
            arr[i].record_cap = int(rec[1])
        if outputs is not None:
            o = outputs[i]
            keep["out"].append(o)
            arr[i].d_snap = o[0].data_ptr() if o[0].numel() else None
            arr[i].d_n_events = o[1].data_ptr() if o[1].numel() else None
            arr[i].d_t_last = o[2].data_ptr() if o[2].numel() else None
            arr[i].d_status = o[3].data_ptr() if o[3].numel() else None
            if len(o) > 4:
                arr[i].d_rec_t = o[4].data_ptr() if o[4].numel() else None
                arr[i].d_rec_j = o[5].data_ptr() if o[5].numel() else None
                arr[i].d_rec_n = o[6].data_ptr() if o[6].numel() else None
    ts = np.ascontiguousarray(snap_t, dtype=np.float64)
    keep["arrays"] += [ts, arr]
    fmt, acc, rnd, norm = parse_mode(mode)
    d = ssa_run_desc()
    d.items = ctypes.addressof(arr)
    d.n_items = len(items)
    d.n_snap = ts.size
    d.t_end = float(t_end)
    d.snap_t = ts.ctypes.data if ts.size else None
    d.seed = int(seed) & (2**64 - 1)
    d.traj_id_base = int(traj_id_base)
    d.format, d.accum, d.rounding, d.norm = fmt, acc, rnd, norm
    d.n_chunks = int(n_chunks)
    d.max_events = int(max_events)
    d.hip_stream = stream
    d.block_size = int(block_size)
    d.grid_size = int(grid_size)
    d.reorder = int(reorder)
    d.first_window = int(first_window)
    d.placement = int(placement)
    return d, keep


(PLACE_AUTO, PLACE_EXPLICIT, PLACE_NEIGHBOUR_PRODUCER, PLACE_WAVE_MAJOR, PLACE_SOLO_WAVE0,
 PLACE_FEED_WAVE0, PLACE_PRODUCER_FIRST, PLACE_DEDICATED_FEED0, PLACE_TWO_FEED0) = 0, 1, 2, 4, 8, 16, 32, 64, 128


def ssa_ensemble_run(items, t_end, snap_t, seed, mode, *, max_events=0, traj_id_base=0, n_chunks=1,
                     block_size=0, grid_size=0, reorder=0, first_window=0, placement=0,
                     torch_outputs=True) -> Run:
    """Queue an ensemble run on torch's current stream. With torch_outputs the
    device outputs are torch tensors owned by the returned Run."""
    import torch
    K = int(np.size(snap_t))
    outputs = None
    if torch_outputs:
        dev = torch.device("cuda", torch.cuda.current_device())
        outputs = []
        for it in items:
            N, E = it["model"].n_species, int(it["n_traj"])
            o = (torch.empty((K, N, E), dtype=torch.int32, device=dev),
                 torch.empty(E, dtype=torch.int64, device=dev),
                 torch.empty(E, dtype=torch.float64, device=dev),
                 torch.empty(E, dtype=torch.uint8, device=dev))
            rec = it.get("record")
            if rec is not None and int(rec[0]) and int(rec[1]) > 0:
                cap = int(rec[1])
                o = o + (torch.empty((E, cap), dtype=torch.float64, device=dev),
                         torch.empty((E, cap), dtype=torch.uint8, device=dev),
                         torch.empty(E, dtype=torch.int32, device=dev))
            outputs.append(o)
    stream = torch.cuda.current_stream().cuda_stream
    d, keep = _desc(items, t_end, snap_t, seed, mode, max_events=max_events, traj_id_base=traj_id_base,
                    n_chunks=n_chunks, block_size=block_size, grid_size=grid_size, reorder=reorder,
                    first_window=first_window, placement=placement, stream=stream, outputs=outputs)
    h = ctypes.c_void_p()
    _check(lib().ssa_ensemble_run(ctypes.byref(d), ctypes.byref(h)))
    meta = [(it["model"].n_species, int(it["n_traj"]), K) for it in items]
    caps = [int(it["record"][1]) if it.get("record") is not None and int(it["record"][0]) else 0 for it in items]
    return Run(h, meta, keep, caps)


def ssa_ensemble_run_noalloc(items, t_end, snap_t, seed, mode, outputs, **kw):
    """Queue a run that allocates no device memory on torch's current stream.
    outputs: per item a tuple of caller-owned device tensors (snap [K, N, E]
    int32, n_events [E] int64, t_last [E] float64, status [E] uint8, and for
    a recording item rec_t, rec_j, rec_n). The kernel must have been loaded by
    an earlier ssa_ensemble_run of the same networks and precision."""
    import torch
    d, keep = _desc(items, t_end, snap_t, seed, mode, stream=torch.cuda.current_stream().cuda_stream,
                    outputs=outputs, **kw)
    _check(lib().ssa_ensemble_run_noalloc(ctypes.byref(d)))
    return keep


def ssa_autotune(items, t_end, snap_t, seed, mode, **kw) -> dict:
    """Time candidate launch shapes on this workload; the best is cached and used
    by later runs that leave block_size / grid_size / n_chunks at 0."""
    import torch
    d, keep = _desc(items, t_end, snap_t, seed, mode, stream=torch.cuda.current_stream().cuda_stream, **kw)
    res = ssa_tune_result()
    _check(lib().ssa_autotune(ctypes.byref(d), ctypes.byref(res)))
    return {f: getattr(res, f) for f, _ in ssa_tune_result._fields_}


def ssa_prepare(items, t_end, snap_t, mode, **kw):
    """Compile and cache the kernel for a run description (no GPU needed)."""
    d, keep = _desc(items, t_end, snap_t, 0, mode, **kw)
    _check(lib().ssa_prepare(ctypes.byref(d)))


def ssa_kernel_file(items, t_end, snap_t, mode, **kw) -> str:  # noqa: D401
    """Path of the cached code object a run description uses (compiles if needed)."""
    d, keep = _desc(items, t_end, snap_t, 0, mode, **kw)
    buf = ctypes.create_string_buffer(4096)
    _check(lib().ssa_kernel_file(ctypes.byref(d), buf, len(buf)))
    return buf.value.decode()


def ssa_dump_source(items, t_end, snap_t, mode, path, **kw):
    d, keep = _desc(items, t_end, snap_t, 0, mode, **kw)
    _check(lib().ssa_dump_source(ctypes.byref(d), str(path).encode()))


def items_from_workload(W, models=None):
    """Binding items for a workloads.Workload (models: optional cache of Model handles)."""
    out = []
    for it in W.items:
        m = models.get(it.model.name) if models is not None else None
        if m is None:
            m = Model(it.model)
            if models is not None:
                models[it.model.name] = m
        d = {"model": m, "x0": it.x0, "n_traj": it.n_traj}
        if it.set_rate is not None:
            d["set_rates"] = it.set_rate
            d["traj_per_set"] = it.traj_per_set
        out.append(d)
    return out
