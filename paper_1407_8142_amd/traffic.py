"""Measure HBM traffic of the level-pass kernels (one or two levels per launch)
with rocprofv3 counters.

Runs four counter passes, each its own rocprofv3 process (one counter group
per run): FETCH_SIZE and WRITE_SIZE of the streaming-copy probe (known bytes:
the calibration), then FETCH_SIZE and WRITE_SIZE of the benchmark.  Each
counter reads KiB per dispatch; dividing by the probe's reading per known
byte gives calibrated bytes.  Writes a JSON entry keyed by workload, tagged
with the SHA-256 of the level-pass sources so that a stale entry is ignored.

    python -m paper_1407_8142_amd.traffic --workload text256 --out DIR
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PROBE = os.path.join(HERE, "bw_probe")
LEVEL_PASS_SOURCES = [os.path.join(HERE, "csrc", f)
                      for f in ("wt_build.hip", "wt_kernels.hpp", "wt_device.hpp", "wt_pair.hpp", "wt_stats.hpp")]
PROBE_MIB = 1024


def source_sha() -> str:
    h = hashlib.sha256()
    for p in LEVEL_PASS_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def run_pass(counter: str, cmd: list[str], out_dir: str, tag: str) -> dict:
    d = os.path.join(out_dir, tag)
    os.makedirs(d, exist_ok=True)
    full = ["timeout", "-s", "KILL", "240", "rocprofv3", "--pmc", counter, "-d", d, "-o", "run",
            "--output-format", "csv", "--", *cmd]
    print("[traffic]", " ".join(full), flush=True)
    env = dict(os.environ, TMPDIR="/tmp")
    with open(os.path.join(out_dir, tag + ".log"), "w") as log:
        subprocess.run(full, check=True, stdout=log, stderr=subprocess.STDOUT, cwd="/tmp", env=env)
    per_kernel = collections.defaultdict(list)
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                per_kernel[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return per_kernel


def is_level_pass(kernel: str) -> bool:
    """One level per launch (level_pass*) or two (pair_pass)."""
    return "level_pass" in kernel or "pair_pass" in kernel


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="text256")
    ap.add_argument("--out", required=True, help="directory for raw rocprofv3 output and the JSON")
    args = ap.parse_args()
    args.out = os.path.abspath(args.out)  # rocprofv3 runs from /tmp
    os.makedirs(args.out, exist_ok=True)
    probe_cmd = [PROBE, str(PROBE_MIB), "3"]
    bench_cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--workload", args.workload, "--steps", "2",
                 "--warmup", "1", "--no-cpu-baseline", "--no-batch", "--no-serve", "--no-matrix", "--no-alphabets"]
    known = PROBE_MIB * 1024.0  # KiB read and written by one copy launch
    cf = run_pass("FETCH_SIZE", probe_cmd, args.out, "copy_fetch")
    cw = run_pass("WRITE_SIZE", probe_cmd, args.out, "copy_write")
    copy_f = [v for k, vs in cf.items() if "copy_u4" in k for v in vs]
    copy_w = [v for k, vs in cw.items() if "copy_u4" in k for v in vs]
    f_scale = known / (sum(copy_f) / len(copy_f))  # true KiB per counted KiB
    w_scale = known / (sum(copy_w) / len(copy_w))
    bf = run_pass("FETCH_SIZE", bench_cmd, args.out, "lp_fetch")
    bw = run_pass("WRITE_SIZE", bench_cmd, args.out, "lp_write")
    kernels = {}
    for k in sorted(set(bf) | set(bw)):
        if not is_level_pass(k) and not any(x in k for x in ("histogram", "stats_prep", "stats_scan", "level_dirs")):
            continue
        f = bf.get(k, [0.0])
        w = bw.get(k, [0.0])
        kernels[k] = {"launches": len(f), "fetch_kib_raw": sum(f) / len(f), "write_kib_raw": sum(w) / len(w),
                      "fetch_bytes": sum(f) / len(f) * f_scale * 1024, "write_bytes": sum(w) / len(w) * w_scale * 1024}
    lp = [(v["launches"], v["fetch_bytes"] + v["write_bytes"]) for k, v in kernels.items() if is_level_pass(k)]
    total_launches = sum(c for c, _ in lp)
    per_launch = sum(c * b for c, b in lp) / total_launches if total_launches else None
    entry = {"source_sha256": source_sha(), "calibration": {"fetch_scale": f_scale, "write_scale": w_scale,
             "probe_bytes_each_way": PROBE_MIB << 20}, "kernels": kernels,
             "traffic_bytes_per_launch": per_launch}
    path = os.path.join(args.out, "traffic_level_pass.json")
    doc = json.load(open(path)) if os.path.exists(path) else {}
    doc[args.workload] = entry
    json.dump(doc, open(path, "w"), indent=1, sort_keys=True)
    print(json.dumps({args.workload: {"traffic_bytes_per_launch": per_launch, "fetch_scale": f_scale,
                                      "write_scale": w_scale}}), flush=True)


if __name__ == "__main__":
    main()
