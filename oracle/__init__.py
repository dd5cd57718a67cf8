"""CPU oracle for the ensemble Gillespie direct method in reduced precision.

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It is the plain,
slow statement of what the GPU path computes (``ssa_oracle.c`` holds the
arithmetic and cites the paper section of every step), and it shares no code
with the GPU library.

Models are passed as any object with the attributes ``n_species``,
``n_reactions``, ``order`` and ``nu`` (M x N int arrays), ``law`` (M ints:
0 mass action, 1 Hill repression, 2 Hill activation), ``rate`` (M floats:
mass-action k_j or Hill v_j) and ``hill_reg``, ``hill_h``, ``hill_b``,
``hill_K`` (M each). Precision modes are named by strings:
``FP64``, ``FP32``, ``{MIX,UNI}_{F16,BF16}_{RTN,SR}`` and, for uniform mode,
a ``_NORM`` suffix (running-max propensity normalisation).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ssa_oracle.c")
_LIB = os.path.join(_HERE, "libssa_oracle.so")

STATUS_NAMES = ("DONE", "ABSORBED", "OVERFLOW", "CAPPED")
FMT_FP64, FMT_FP32, FMT_FP16, FMT_BF16 = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with FMA contraction off (binary32/64 ops stay
    single correctly rounded IEEE operations)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", *_arch_flags(),
               "-fopenmp", "-shared", "-fPIC", "-Wall", "-Wextra", "-Wno-maybe-uninitialized", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


class _Model(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("n_reactions", ctypes.c_int32),
                ("order", ctypes.c_void_p), ("nu", ctypes.c_void_p), ("law", ctypes.c_void_p),
                ("rate", ctypes.c_void_p), ("hill_reg", ctypes.c_void_p), ("hill_h", ctypes.c_void_p),
                ("hill_b", ctypes.c_void_p), ("hill_K", ctypes.c_void_p)]


class _Mode(ctypes.Structure):
    _fields_ = [("fmt", ctypes.c_int32), ("uniform", ctypes.c_int32), ("sr", ctypes.c_int32),
                ("norm", ctypes.c_int32)]


class _Rec(ctypes.Structure):
    _fields_ = [("mask", ctypes.c_uint64), ("cap", ctypes.c_int32), ("t", ctypes.c_void_p),
                ("j", ctypes.c_void_p), ("n", ctypes.c_void_p)]


class _Run(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_void_p), ("t_end", ctypes.c_double), ("snap_t", ctypes.c_void_p),
                ("n_snap", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("traj_id_base", ctypes.c_uint32), ("max_events", ctypes.c_uint64),
                ("set_rate", ctypes.c_void_p), ("n_sets", ctypes.c_int64),
                ("traj_per_set", ctypes.c_int64)]


_lib = None


def _arch_flags():
    """-mfma where the host has FMA3, so the explicit fma()/fmaf() calls of the
    logarithm are single instructions (the same correctly rounded operation as
    libm's, which emulates it otherwise); contraction stays off."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("flags") and " fma " in line + " ":
                    return ["-mfma"]
    except OSError:
        pass
    return []


def build_variant(src_text: str, out_path: str) -> str:
    """Compile oracle source text (e.g. a deliberately altered copy used by the
    tests that check the pins catch mistakes) into out_path."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", *_arch_flags(), "-fopenmp",
                    "-shared", "-fPIC", "-w", "-o", out_path, src, "-lm"], check=True)
    return out_path


def _open(path):
    lib = ctypes.CDLL(path)
    lib.or_simulate.restype = ctypes.c_int
    lib.or_simulate.argtypes = [ctypes.POINTER(_Model), _Mode, ctypes.POINTER(_Run),
                                ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.POINTER(_Rec), ctypes.c_int32]
    for name in ("or_philox_batch", "or_nlog64_batch", "or_nlog32_batch", "or_uniform_batch"):
        getattr(lib, name).restype = None
    lib.or_round16_batch.restype = None
    lib.or_sr_field_batch.restype = None
    lib.or_sr_field_batch.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
    lib.or_round16_batch.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int64]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _open(_LIB)
    return _lib


@dataclass(frozen=True)
class Mode:
    fmt: int
    uniform: bool = False
    sr: int = 0          # 0 round to nearest, 1 SR at every op, 2 SR at accumulation points
    norm: bool = False


def parse_mode(name: str) -> Mode:
    """Parse FP64 / FP32 / {MIX,UNI}_{F16,BF16}_{RTN,SR}[_NORM] / UNI_{F16,BF16}_SRA[_NORM]
    (SRA: stochastic rounding only at the partial sums and the clock)."""
    if name == "FP64":
        return Mode(FMT_FP64)
    if name == "FP32":
        return Mode(FMT_FP32)
    parts = name.split("_")
    if len(parts) not in (3, 4) or parts[0] not in ("MIX", "UNI") or parts[1] not in ("F16", "BF16") \
            or parts[2] not in ("RTN", "SR", "SRA") or (len(parts) == 4 and (parts[3] != "NORM" or parts[0] != "UNI")) \
            or (parts[2] == "SRA" and parts[0] != "UNI"):
        raise ValueError(f"unknown precision mode {name!r}")
    return Mode(FMT_FP16 if parts[1] == "F16" else FMT_BF16, parts[0] == "UNI",
                {"RTN": 0, "SR": 1, "SRA": 2}[parts[2]], len(parts) == 4)


def _ptr(a):
    return None if a is None else a.ctypes.data


def simulate(model, mode: str, x0, t_end: float, snap_t, seed: int, *, n_traj: int | None = None,
             indices=None, traj_id_base: int = 0, max_events: int = 0, set_rate=None,
             traj_per_set: int = 0, threads: int = 1, record_mask: int = 0, record_cap: int = 0, lib=None):
    """Run trajectories ``indices`` (default ``range(n_traj)``) of an ensemble.

    Returns a dict with ``snap`` [K, N, count] int32, ``n_events`` uint64,
    ``t_last`` float64 and ``status`` uint8 per trajectory; with a non-zero
    ``record_mask`` (bit j: reaction j) also the event record: ``rec_t``
    [count, record_cap] float64 (clock after each recorded firing), ``rec_j``
    [count, record_cap] uint8 (reaction) and ``rec_n`` uint32 (recorded
    firings, also those past ``record_cap``). ``lib``: a library from
    ``_open`` (default: the built oracle).
    """
    lib = lib or _load()
    if indices is None:
        indices = np.arange(int(n_traj), dtype=np.int64)
    idx = np.ascontiguousarray(indices, dtype=np.int64)
    N, M = int(model.n_species), int(model.n_reactions)
    keep = []

    def arr(a, dt):
        b = np.ascontiguousarray(a, dtype=dt)
        keep.append(b)
        return b

    order = arr(model.order, np.int32).reshape(M, N)
    nu = arr(model.nu, np.int32).reshape(M, N)
    law = arr(model.law, np.int32)
    rate = arr(model.rate, np.float64)
    hr, hh = arr(model.hill_reg, np.int32), arr(model.hill_h, np.int32)
    hb, hK = arr(model.hill_b, np.float64), arr(model.hill_K, np.float64)
    md = _Model(N, M, _ptr(order), _ptr(nu), _ptr(law), _ptr(rate), _ptr(hr), _ptr(hh), _ptr(hb), _ptr(hK))
    m = parse_mode(mode)
    cm = _Mode(m.fmt, int(m.uniform), int(m.sr), int(m.norm))
    x0a = arr(x0, np.int32)
    ts = arr(snap_t, np.float64)
    sr_tab = None if set_rate is None else arr(set_rate, np.float64)
    n_sets = 0 if sr_tab is None else sr_tab.size // M
    run = _Run(_ptr(x0a), float(t_end), _ptr(ts), ts.size, int(seed) & (2**64 - 1),
               int(traj_id_base), int(max_events), _ptr(sr_tab), n_sets, int(traj_per_set))
    count = idx.size
    K = ts.size
    snap = np.zeros((K, N, count), dtype=np.int32)
    n_ev = np.zeros(count, dtype=np.uint64)
    t_last = np.zeros(count, dtype=np.float64)
    status = np.zeros(count, dtype=np.uint8)
    out = {"snap": snap, "n_events": n_ev, "t_last": t_last, "status": status}
    rec = None
    if record_mask:
        cap = int(record_cap)
        out["rec_t"] = np.zeros((count, cap), dtype=np.float64)
        out["rec_j"] = np.zeros((count, cap), dtype=np.uint8)
        out["rec_n"] = np.zeros(count, dtype=np.uint32)
        rec = _Rec(int(record_mask) & (2**64 - 1), cap, _ptr(out["rec_t"]), _ptr(out["rec_j"]), _ptr(out["rec_n"]))
    rc = lib.or_simulate(ctypes.byref(md), cm, ctypes.byref(run), _ptr(idx), count, _ptr(snap),
                         _ptr(n_ev), _ptr(t_last), _ptr(status), ctypes.byref(rec) if rec else None,
                         int(threads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out


def sr_fields(fmt: str, seed: int, ids, ns, slots, conv, lib=None):
    """The SR random halfwords (field << (16 - B)) the 16-bit trajectory code
    reads for main (conv = 0) or conversion (conv = 1) slots; fmt 'F16' or 'BF16'."""
    lib = lib or _load()
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    ns = np.ascontiguousarray(ns, dtype=np.uint64)
    sl = np.ascontiguousarray(slots, dtype=np.int32)
    cv = np.ascontiguousarray(conv, dtype=np.int32)
    out = np.empty(ids.size, dtype=np.int32)
    lib.or_sr_field_batch(ctypes.c_int(2 if fmt == "F16" else 3), ctypes.c_uint64(int(seed) & (2**64 - 1)),
                          _ptr(ids), _ptr(ns), _ptr(sl), _ptr(cv), _ptr(out), ctypes.c_int64(ids.size))
    return out


def philox(ctr, key, lib=None):
    """Philox4x32-10 of counters ctr [n,4] under keys key [n,2] -> [n,4] uint32."""
    lib = lib or _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.empty_like(c)
    lib.or_philox_batch(ctypes.c_void_p(c.ctypes.data), ctypes.c_void_p(k.ctypes.data),
                        ctypes.c_void_p(out.ctypes.data), ctypes.c_int64(c.shape[0]))
    return out


def nlog64(u, lib=None):
    """-ln(u), FP64 project logarithm, for u in (0, 1]."""
    lib = lib or _load()
    a = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(a)
    lib.or_nlog64_batch(ctypes.c_void_p(a.ctypes.data), ctypes.c_void_p(out.ctypes.data), ctypes.c_int64(a.size))
    return out


def nlog32(u, lib=None):
    """-ln(u), FP32 project logarithm, for u in (0, 1]."""
    lib = lib or _load()
    a = np.ascontiguousarray(u, dtype=np.float32)
    out = np.empty_like(a)
    lib.or_nlog32_batch(ctypes.c_void_p(a.ctypes.data), ctypes.c_void_p(out.ctypes.data), ctypes.c_int64(a.size))
    return out


def round16(fmt: int, v, rb=None, lib=None):
    """Round doubles to fp16 (fmt=2) or bf16 (fmt=3): RNE, or SR with halfwords rb."""
    lib = lib or _load()
    a = np.ascontiguousarray(v, dtype=np.float64)
    r = None if rb is None else np.ascontiguousarray(np.broadcast_to(rb, a.shape), dtype=np.int32)
    out = np.empty_like(a)
    lib.or_round16_batch(int(fmt), a.ctypes.data, None if r is None else r.ctypes.data,
                         out.ctypes.data, a.size)
    return out


def uniforms(w, lib=None):
    """(u53 from word pairs, u24 from the first word of each pair) for w [n,2]."""
    lib = lib or _load()
    a = np.ascontiguousarray(w, dtype=np.uint32).reshape(-1, 2)
    u53 = np.empty(a.shape[0], dtype=np.float64)
    u24 = np.empty(a.shape[0], dtype=np.float32)
    lib.or_uniform_batch(ctypes.c_void_p(a.ctypes.data), ctypes.c_void_p(u53.ctypes.data),
                         ctypes.c_void_p(u24.ctypes.data), ctypes.c_int64(a.shape[0]))
    return u53, u24
