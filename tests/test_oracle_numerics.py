"""Pins of the oracle's numeric building blocks against things other than
itself: published known-answer vectors, an independent Philox implementation
(rocRAND's), arbitrary-precision logarithms, numpy/torch IEEE conversions and
brute-force enumeration of the 16-bit grids."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v, 16) for v in line.split()])
    return np.array(rows, dtype=np.uint64).astype(np.uint32)


def test_philox_known_answers(orc):
    kat = _kat()
    out = orc.philox(kat[:, 0:4], kat[:, 4:6])
    np.testing.assert_array_equal(out, kat[:, 6:10])


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_engine(orc, tmp_path):
    """rocRAND's host-callable Philox4x32-10 rounds as an independent implementation."""
    src = tmp_path / "rr.cpp"
    src.write_text(
        "#include <rocrand/rocrand_philox4x32_10.h>\n#include <cstdio>\n"
        "struct E : rocrand_device::philox4x32_10_engine { uint4 r(uint4 c, uint2 k) { return ten_rounds(c, k); } };\n"
        "int main() { E e; unsigned a,b,c,d,k0,k1;\n"
        " while (scanf(\"%x %x %x %x %x %x\", &a,&b,&c,&d,&k0,&k1) == 6) {\n"
        "  uint4 o = e.r(uint4{a,b,c,d}, uint2{k0,k1}); printf(\"%08x %08x %08x %08x\\n\", o.x,o.y,o.z,o.w); } }\n")
    exe = tmp_path / "rr"
    subprocess.run(["hipcc", "-O1", str(src), "-o", str(exe)], check=True, capture_output=True)
    rng = np.random.default_rng(11)
    ctr = rng.integers(0, 2**32, size=(500, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(500, 2), dtype=np.uint64).astype(np.uint32)
    inp = "\n".join(" ".join(f"{v:x}" for v in list(c) + list(k)) for c, k in zip(ctr, key))
    res = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
    ref = np.array([[int(v, 16) for v in ln.split()] for ln in res.stdout.strip().splitlines()],
                   dtype=np.uint64).astype(np.uint32)
    np.testing.assert_array_equal(orc.philox(ctr, key), ref)


def test_uniforms_exact_and_in_unit_interval(orc):
    rng = np.random.default_rng(3)
    w = rng.integers(0, 2**32, size=(100000, 2), dtype=np.uint64).astype(np.uint32)
    w = np.vstack([w, [[0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [0, 0x7FF], [0xFFFFFFFF, 0]]]).astype(np.uint32)
    u53, u24 = orc.uniforms(w)
    assert np.all(u53 > 0) and np.all(u53 <= 1) and np.all(u24 > 0) and np.all(u24 <= 1)
    m53 = (w[:, 0].astype(np.uint64) << np.uint64(21)) | (w[:, 1].astype(np.uint64) >> np.uint64(11))
    # u * 2^53 is the integer m + 1 exactly
    np.testing.assert_array_equal(np.ldexp(u53, 53).astype(np.uint64), m53 + np.uint64(1))
    np.testing.assert_array_equal(np.ldexp(u24.astype(np.float64), 24).astype(np.uint64),
                                  (w[:, 0] >> 8).astype(np.uint64) + 1)
    assert u53[-4] == 2.0 ** -53 and u53[-3] == 1.0 and u24[-3] == 1.0 and u24[-4] == 2.0 ** -24


def _ulp_err_mp(vals, ref_fn, dtype):
    import mpmath
    mpmath.mp.prec = 120
    errs = []
    for v, got in vals:
        exact = ref_fn(v)
        ulp = float(np.spacing(dtype(abs(float(exact))))) if exact != 0 else float(np.finfo(dtype).tiny)
        errs.append(abs(float(mpmath.mpf(float(got)) - exact)) / ulp)
    return max(errs)


def test_nlog64_vs_mpmath(orc):
    import mpmath
    mpmath.mp.prec = 120
    rng = np.random.default_rng(5)
    m = rng.integers(0, 2**53, size=20000, dtype=np.uint64)
    u = (m.astype(np.float64) + 1.0) * 2.0 ** -53
    u = np.concatenate([u, 2.0 ** -np.arange(0, 54, dtype=np.float64),
                        1 - 2.0 ** -np.arange(1, 54, dtype=np.float64),
                        [0.70710678118654746, 0.70710678118654757, 0.5000000000000001, 0.9999999]])
    got = orc.nlog64(u)
    assert orc.nlog64(np.array([1.0]))[0] == 0.0
    assert math.copysign(1.0, orc.nlog64(np.array([1.0]))[0]) == 1.0
    worst = _ulp_err_mp(zip(u.tolist(), got.tolist()), lambda v: -mpmath.log(mpmath.mpf(v)), np.float64)
    assert worst <= 2.0, worst


def test_nlog32_vs_mpmath(orc):
    import mpmath
    mpmath.mp.prec = 80
    rng = np.random.default_rng(6)
    m = rng.integers(0, 2**24, size=20000)
    u = ((m + 1) * 2.0 ** -24).astype(np.float32)
    u = np.concatenate([u, (2.0 ** -np.arange(0, 25)).astype(np.float32),
                        (1 - 2.0 ** -np.arange(1, 25)).astype(np.float32)])
    got = orc.nlog32(u)
    assert orc.nlog32(np.array([1.0], np.float32))[0] == 0.0
    worst = _ulp_err_mp(zip(u.astype(np.float64).tolist(), got.astype(np.float64).tolist()),
                        lambda v: -mpmath.log(mpmath.mpf(v)), np.float32)
    assert worst <= 2.0, worst


def _f32_probe_values():
    """All 2^16 high halves of binary32 combined with low halves that sit on
    and around every rounding boundary of fp16 (13 dropped bits) and bf16 (16)."""
    hi = np.arange(0, 1 << 16, dtype=np.uint32) << np.uint32(16)
    lows = np.array([0, 1, 0x0FFF, 0x1000, 0x1001, 0x1FFF, 0x2000, 0x3000, 0x5000, 0x7FFF, 0x8000,
                     0x8001, 0x9000, 0xD000, 0xEFFF, 0xF000, 0xFFFF], dtype=np.uint32)
    bits = (hi[:, None] | lows[None, :]).ravel()
    rng = np.random.default_rng(8)
    bits = np.concatenate([bits, rng.integers(0, 2**32, size=300000, dtype=np.uint64).astype(np.uint32)])
    return bits.view(np.float32)


def test_round16_rne_fp16_matches_numpy(orc):
    x = _f32_probe_values()
    got = orc.round16(orc.FMT_FP16, x.astype(np.float64))
    ref = x.astype(np.float16).astype(np.float64)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    np.testing.assert_array_equal(got[~nan], ref[~nan])
    # signed zeros preserved
    assert np.array_equal(np.signbit(got[~nan]), np.signbit(ref[~nan]))


def test_round16_rne_fp16_from_double_matches_numpy(orc):
    rng = np.random.default_rng(9)
    v = np.concatenate([rng.uniform(0, 70000, 100000), np.exp(rng.uniform(-25, 11, 100000)),
                        [65504.0, 65519.999, 65520.0, 65536.0, 2.0 ** -25, 2.0 ** -25 * 1.0000001,
                         1.5e-5, 1.6666666666666667e-05]])
    got = orc.round16(orc.FMT_FP16, v)
    np.testing.assert_array_equal(got, v.astype(np.float16).astype(np.float64))


def test_round16_rne_bf16_matches_torch(orc):
    torch = pytest.importorskip("torch")
    x = _f32_probe_values()
    got = orc.round16(orc.FMT_BF16, x.astype(np.float64))
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).to(torch.float64).numpy()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    np.testing.assert_array_equal(got[~nan], ref[~nan])


def _grid(fmt):
    """All finite non-negative values of the 16-bit format, ascending (brute force)."""
    import torch
    b = np.arange(0, 0x7C00 if fmt == 2 else 0x7F80, dtype=np.uint16)
    if fmt == 2:
        return b.view(np.float16).astype(np.float64)
    return torch.from_numpy(b.view(np.int16).copy()).view(torch.bfloat16).to(torch.float64).numpy()


@pytest.mark.parametrize("fmt", [2, 3])
def test_round16_rne_from_double_is_nearest_grid_point(orc, fmt):
    pytest.importorskip("torch")
    g = _grid(fmt)
    rng = np.random.default_rng(10 + fmt)
    v = np.exp(rng.uniform(np.log(g[1]) - 1, np.log(g[-1]), 50000))
    v = v[v < g[-1]]
    got = orc.round16(fmt, v)
    i = np.searchsorted(g, v, side="right") - 1
    lo, hi = g[i], g[np.minimum(i + 1, g.size - 1)]
    dl, dh = v - lo, hi - v
    even_lo = (i % 2) == 0
    ref = np.where(dl < dh, lo, np.where(dh < dl, hi, np.where(even_lo, lo, hi)))
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("fmt", [2, 3])
def test_sr_neighbours_and_unbiased(orc, fmt):
    """SR (Sec. 3.3): every outcome is one of the two bracketing grid points, and
    over all 2^16 halfwords the mean equals x to within a 2^-B fraction of the
    grid step (B = 13 random bits for fp16, 16 for bf16); exact grid points
    never move."""
    pytest.importorskip("torch")
    g = _grid(fmt)
    rng = np.random.default_rng(20 + fmt)
    top = 60000.0 if fmt == 2 else 1e30
    xs = np.exp(rng.uniform(np.log(1e-7), np.log(top), 200)).astype(np.float32).astype(np.float64)
    xs = np.concatenate([xs, g[[1, 5, 700, 1000, 3000]]])
    rb = np.arange(65536, dtype=np.int32)
    for x in xs:
        out = orc.round16(fmt, np.full(65536, x), rb)
        i = np.searchsorted(g, x, side="right") - 1
        lo = g[i]
        hi = g[i + 1] if i + 1 < g.size else np.inf
        assert set(np.unique(out)).issubset({lo, hi})
        if x == lo:
            assert np.all(out == lo)
            continue
        B = 13 if fmt == 2 else 16
        mean = lo + (hi - lo) * np.count_nonzero(out == hi) / 65536.0
        assert abs(mean - x) <= (hi - lo) / 2.0 ** B * (1 + 1e-12)
        # probability of rounding up is (x - lo) / (hi - lo), quantised down to 2^-B
        p_up = np.count_nonzero(out == hi) / 65536.0
        assert 0 <= (x - lo) / (hi - lo) - p_up < 2.0 ** -B
        # the decision depends only on the top B bits of the halfword
        np.testing.assert_array_equal(out.reshape(2 ** B, -1), np.repeat(out[:: 2 ** (16 - B), None], 2 ** (16 - B), 1))


def test_sr_overflow_to_infinity(orc):
    # between the largest finite fp16 (65504) and 2^16, SR rounds up to +inf
    out = orc.round16(2, np.full(65536, 65520.0), np.arange(65536, dtype=np.int32))
    assert np.count_nonzero(np.isinf(out)) == 32768 and np.all((out == 65504.0) | np.isinf(out))
    assert np.isinf(orc.round16(2, np.array([70000.0]), np.array([0]))[0])
    assert np.isinf(orc.round16(2, np.array([65520.0]))[0])  # RNE tie goes to even = overflow


@pytest.mark.parametrize("fmt", [2, 3])
def test_binary32_op_then_round_is_correctly_rounded_16bit_op(orc, fmt):
    """Double rounding is innocuous when the wide format has >= 2p+2 bits
    (Figueroa): rounding the binary32 result of +, -, *, / on 16-bit operands
    equals rounding the (much more precise) binary64 result."""
    pytest.importorskip("torch")
    g = _grid(fmt)
    if fmt == 3:
        g = g[(g > 2.0 ** -60) & (g < 2.0 ** 60)]   # keep bf16 products finite and normal
    rng = np.random.default_rng(30 + fmt)
    a = g[rng.integers(1, g.size, 40000)] * rng.choice([1.0, -1.0], 40000)
    b = g[rng.integers(1, g.size, 40000)]
    for op in (np.add, np.subtract, np.multiply, np.divide):
        with np.errstate(all="ignore"):
            wide = op(a, b)
            narrow = op(a.astype(np.float32), b.astype(np.float32)).astype(np.float64)
        ok = np.isfinite(wide)
        np.testing.assert_array_equal(orc.round16(fmt, narrow[ok]), orc.round16(fmt, wide[ok]))
