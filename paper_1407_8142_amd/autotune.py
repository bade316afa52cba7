"""Autotuner of the batched build's launch: times wt_batch_run under each
candidate wt_tune on the batch itself and keeps the fastest.

The tunables are the launch form (one persistent launch over the whole
queue, or one launch per phase), the resident blocks per CU of the work
kernel, and the work items taken per queue access.  The tile shape (16 KiB
per tile, 256 threads) is fixed by the kernels.  Every candidate produces
the same outputs (the tests check this), so only time decides.
"""
from __future__ import annotations

import json
import os

import torch

from . import wt

DEFAULT_CANDIDATES = [(mode, bpc, chunk)
                      for mode in (wt.BATCH_PERSISTENT, wt.BATCH_PER_PHASE)
                      for bpc in (0, 4, 2)
                      for chunk in (1, 4)]


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
             key: str | None = None) -> tuple["wt.Tune", list[dict]]:
    """Returns the fastest tune and the table of every candidate's time.
    With `cache_path` and `key`, a previous result for the same key is
    reused and a new one is stored."""
    if cache_path and key and os.path.exists(cache_path):
        try:
            cached = json.load(open(cache_path)).get(key)
        except (OSError, ValueError):
            cached = None
        if cached:
            return wt.Tune(**cached["best"]), cached["table"]
    table = []
    for mode, bpc, chunk in candidates or DEFAULT_CANDIDATES:
        t = wt.Tune(mode=mode, blocks_per_cu=bpc, chunk=chunk)
        ms = time_run(batch, t, reps)
        rc, _ = batch.status()
        if rc != wt.WT_OK:
            raise RuntimeError(f"batch failed under {t.as_dict()}: {wt.STATUS_NAMES.get(rc, rc)}")
        table.append({"tune": t.as_dict(), "ms": round(ms, 4)})
    best = min(table, key=lambda r: r["ms"])
    if cache_path and key:
        try:
            doc = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        except (OSError, ValueError):
            doc = {}
        doc[key] = {"best": best["tune"], "table": table}
        with open(cache_path, "w") as f:
            json.dump(doc, f, indent=1)
    return wt.Tune(**best["tune"]), table
