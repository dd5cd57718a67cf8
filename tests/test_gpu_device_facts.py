"""Exactness facts the simulation kernel relies on, checked on the device
against the kernel's own device functions (tests/gpu_checks.hip includes the
device template):

* gfx950's SR conversions read only the top B bits of their random operand
  (13 for fp16, 16 for bf16), so the kernel may hand a conversion a packed
  word whose low bits belong to other random fields (the rounding rule the
  oracle states, on the field alone, is then unchanged);
* the short fma divisions return the IEEE quotient: div_rn_log on every log
  argument, div_rn_inrange on -ln(u1)/a0 over the fp16 ranges, div_rn_log64
  on 2^31 binary64 log arguments and the ends of both binades, so the kernel's
  logarithms and waiting times equal the oracle's correctly rounded divisions.
"""
import ctypes
import os

import pytest

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgpu_checks.so")


def _lib():
    import torch  # one HIP runtime per process: torch's, loaded first
    assert torch.cuda.is_available()
    if not os.path.exists(LIB):
        pytest.fail("tests/libgpu_checks.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    lib.gpu_check_sr_lowbits.argtypes = [ctypes.c_ulonglong, ctypes.POINTER(ctypes.c_ulonglong)]
    lib.gpu_check_division.argtypes = [ctypes.c_uint, ctypes.c_int, ctypes.POINTER(ctypes.c_ulonglong)]
    lib.gpu_check_division64.argtypes = [ctypes.c_ulonglong, ctypes.POINTER(ctypes.c_ulonglong)]
    return lib


@pytest.mark.gpu
def test_sr_conversions_read_only_top_bits_of_random_operand():
    out = (ctypes.c_ulonglong * 2)()
    n = 1 << 26
    print(f"[gpu-facts] sr low bits, {n} pairs", flush=True)
    assert _lib().gpu_check_sr_lowbits(n, out) == 0
    assert list(out) == [0, 0], f"fp16 / bf16 mismatches: {list(out)}"


@pytest.mark.gpu
def test_short_division_is_ieee_on_its_ranges():
    out = (ctypes.c_ulonglong * 2)()
    print("[gpu-facts] division: every log argument; every 4th numerator x 8 denominators", flush=True)
    assert _lib().gpu_check_division(4, 8, out) == 0
    assert list(out) == [0, 0], f"log-argument / tau mismatches: {list(out)}"


@pytest.mark.gpu
def test_short_binary64_log_division_is_ieee():
    out = (ctypes.c_ulonglong * 1)()
    n = 1 << 30
    print(f"[gpu-facts] binary64 log division: {2 * (n + 128)} arguments", flush=True)
    assert _lib().gpu_check_division64(n, out) == 0
    assert list(out) == [0], f"mismatches: {list(out)}"
