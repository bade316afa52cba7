"""Autotuner of the batched build's launch: times wt_batch_run under each
candidate wt_tune on the batch itself and keeps the fastest.

The tunables are the launch form (one persistent launch over the whole
queue, or one launch per phase), the resident blocks per CU of the work
kernel, the work items taken per queue access, and the levels per LDS pass:
each job's tail levels fused on chip once its nodes fit a segment, at most
the last m of them, or every level a pass of its own (`wt.set_fused_levels`).  The tile shape (16 KiB per
tile, 256 threads, so 16/8/4 symbols per thread at 1/2/4 bytes) is a
compile-time constant of the kernels: their LDS layouts, register tiles and
unrolled loops are sized by it.  Every candidate produces the same outputs
(the tests check this), so only time decides.
"""
from __future__ import annotations

import json
import os

import torch

from . import wt

# (launch form, blocks per CU, chunk, fused tail levels: 0 none, 1 all that
# fit, m >= 2 at most the last m)
DEFAULT_CANDIDATES = ([(wt.BATCH_PERSISTENT, bpc, chunk, 1) for bpc, chunk in ((0, 1), (4, 4))] +
                      [(wt.BATCH_PER_PHASE, bpc, chunk, 1) for bpc, chunk in ((0, 4), (4, 4))] +
                      [(wt.BATCH_PER_PHASE, bpc, 1, fused) for bpc in (0, 4) for fused in (1, 0, 12, 10, 8, 6, 4)])


def time_run(batch: "wt.Batch", tune: "wt.Tune", reps: int = 3) -> float:
    """Median device milliseconds of wt_batch_run under `tune` (after one
    untimed run)."""
    stream = torch.cuda.current_stream()
    batch.run(tune)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        batch.run(tune)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def autotune(batch: "wt.Batch", candidates=None, reps: int = 3, cache_path: str | None = None,
             key: str | None = None) -> tuple["wt.Tune", list[dict], bool]:
    """Returns the fastest tune, the table of every candidate's time, and
    whether that candidate fused the tail levels (this thread's fusion
    setting is left at that value).  With `cache_path` and `key`, a previous
    result for the same key is reused and a new one is stored."""
    if cache_path and key and os.path.exists(cache_path):
        try:
            cached = json.load(open(cache_path)).get(key)
        except (OSError, ValueError):
            cached = None
        if cached:
            wt.set_fused_levels(cached["fused"])
            return wt.Tune(**cached["best"]), cached["table"], cached["fused"]
    table = []
    try:
        for mode, bpc, chunk, fused in candidates or DEFAULT_CANDIDATES:
            wt.set_fused_levels(fused)
            t = wt.Tune(mode=mode, blocks_per_cu=bpc, chunk=chunk)
            ms = time_run(batch, t, reps)
            rc, _ = batch.status()
            if rc != wt.WT_OK:
                raise RuntimeError(f"batch failed under {t.as_dict()}: {wt.STATUS_NAMES.get(rc, rc)}")
            table.append({"tune": t.as_dict(), "fused": fused, "ms": round(ms, 4)})
    finally:
        wt.set_fused_levels(1)
    best = min(table, key=lambda r: r["ms"])
    wt.set_fused_levels(best["fused"])
    if cache_path and key:
        try:
            doc = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        except (OSError, ValueError):
            doc = {}
        doc[key] = {"best": best["tune"], "fused": best["fused"], "table": table}
        with open(cache_path, "w") as f:
            json.dump(doc, f, indent=1)
    return wt.Tune(**best["tune"]), table, best["fused"]
