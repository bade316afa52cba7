"""Compile the HIP sources into the in-tree shared library ``libwt.so`` (gfx950)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwt.so")
PROBE = os.path.join(HERE, "bw_probe")
SOURCES = ["wt_build.hip", "wt_batch.hip", "wt_query.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def hipcc_flags() -> list[str]:
    return [
        "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
        "-Wall", "-Wno-unused-function",
        # Keep the compiler from emitting packed-FP32 instructions.
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
    ]


def build_library(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *hipcc_flags(), "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_probe(verbose: bool = False) -> str:
    """Streaming-copy probe (HBM bandwidth and counter calibration), an executable."""
    flags = [f for f in hipcc_flags() if f not in ("-fPIC", "-shared")]
    cmd = [HIPCC, *flags, "-o", PROBE, os.path.join(CSRC, "bw_probe.hip")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return PROBE


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
    print(build_probe(verbose="-v" in sys.argv))
