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
    """One object per source, compiled in parallel, then one link."""
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        flags = [f for f in hipcc_flags() if f != "-shared"]
        cmd = [HIPCC, *flags, "-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [cmd for cmd, p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-fPIC", "-shared", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    for obj in objs:
        os.remove(obj)
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
