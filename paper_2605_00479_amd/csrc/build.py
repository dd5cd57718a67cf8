"""Build libssa_rp.so (host C ABI + embedded device template) in-tree.

    python -m paper_2605_00479_amd.csrc.build

The device template ssa_device.hip is embedded as a string and compiled per
(networks, precision) combination at run time by hipRTC for gfx950; this step
also compiles it once for a probe network (a syntax check needing no GPU).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libssa_rp.so")
PEAK_LIB = os.path.join(PKG, "libssa_valu_peak.so")

HIP_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def embed_device_source() -> str:
    os.makedirs(BUILD, exist_ok=True)
    with open(os.path.join(HERE, "ssa_device.hip")) as f:
        src = f.read()
    delim = "SSADEV"
    assert ")" + delim + '"' not in src
    out = os.path.join(BUILD, "ssa_device_src.inc")
    text = ("// generated from ssa_device.hip by build.py\n"
            f"static const char kDeviceSource[] = R\"{delim}(\n{src}){delim}\";\n")
    old = open(out).read() if os.path.exists(out) else None
    if old != text:
        with open(out, "w") as f:
            f.write(text)
    return out


def build_library(verbose: bool = False) -> str:
    embed_device_source()
    cmd = ["hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall", *HIP_FLAGS,
           "-I", os.path.join(ROOT, "include"), "-I", BUILD,
           os.path.join(HERE, "ssa_capi.cpp"), "-o", LIB + ".tmp", "-lhiprtc", "-ldl"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("building libssa_rp.so failed")
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    os.replace(LIB + ".tmp", LIB)
    hip_shared(os.path.join(HERE, "valu_peak.hip"), PEAK_LIB)
    return LIB


def hip_shared(src: str, out: str) -> str:
    """Compile one HIP source into a shared library for gfx950."""
    cmd = ["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", *HIP_FLAGS,
           src, "-o", out + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"building {os.path.basename(out)} failed")
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))
