"""Benchmark: one step = one full wt_build (validation + histogram + C +
node tables + every level pass with rank/select directories) of a synthetic
sequence already resident in HBM.

Prints ONE JSON line.  Default workload: text-like n = 2^28 uint8, sigma = 256
(Zipf(1.1) symbols over a permuted byte alphabet, geometric runs of mean 4).
The line also carries a "batch" object: 4096 sequences (lengths
log-uniform in [2^10, 2^20], sigma in {4, 256, 2^16}) built by one
wt_batch_run (autotuned launch, replayed as a captured graph) against one
wt_build per sequence on the same GPU, with the two outputs compared bit
for bit.

A "serve" object reports the serving loop on a Poisson trace (2000 build
requests/s, n log-uniform in [2^12, 2^26], sigma log-uniform in [4, 2^20],
Zipf(1.1) symbols; 100 query batches/s of 10^5 access/rank queries over
the resident trees; 64 GB resident budget with LRU eviction): p50/p99
build and query-batch latency beside throughput.

  python bench.py [--steps K] [--warmup W] [--workload text256|uniform256|alpha16|alpha20]
                  [--no-cpu-baseline] [--no-batch] [--batch-count N] [--no-serve] [--serve-seconds S]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "symbols*levels/s and % HBM peak; batched vs per-seq builds, bit-exact"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_level_pass.json")
LEVEL_PASS_SOURCES = [os.path.join(ROOT, "paper_1407_8142_amd", "csrc", f)
                      for f in ("wt_build.hip", "wt_kernels.hpp", "wt_device.hpp", "wt_pair.hpp", "wt_stats.hpp")]

WORKLOADS = {
    "text256": ("text-like: n=2^28 uint8, sigma=256, Zipf(1.1) over a permuted byte alphabet, geometric runs "
                "(mean 4)", 1 << 28),
    "uniform256": ("uniform: n=2^20 uint8, sigma=256, i.i.d.", 1 << 20),
    "alpha16": ("large alphabet: n=2^27 uint32, sigma=2^16, half uniform, half Zipf(1.0) word-id-like", 1 << 27),
    "alpha20": ("large alphabet: n=2^27 uint32, sigma=2^20, half uniform, half Zipf(1.0) word-id-like", 1 << 27),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_sha() -> str:
    h = hashlib.sha256()
    for p in LEVEL_PASS_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def level_pass_bytes(n: int, L: int, in_bytes: int, mid_bytes: int, passes: int,
                     lastbits: bool = False) -> list[float]:
    """Algorithmic HBM bytes of each level-pass launch.  One level per pass:
    read the level's sequence, write the next one (not on the last level),
    write the level bits (n/8), the rank directory (8 B per 512 bits) and
    select samples (8 B per 4096 ones and per 4096 zeros).  With `lastbits`
    level L-2 writes the last level's bits (n/8) instead of its sequence,
    and the last launch reads those bits (n/8) for the directories.  Two
    levels per pass (byte alphabets): read S_l once, write S_{l+2} (not from
    the last pair), and two levels of bits and directories; an odd last
    level alone."""
    dirs = n / 8 + n / 64 + n / 256
    out = []
    if passes == L:
        for l in range(L):
            rd = in_bytes if l == 0 else mid_bytes
            wr = mid_bytes if l + 1 < L else 0
            if lastbits and l + 2 == L:
                out.append(n * rd + dirs + n / 8)
            elif lastbits and l + 1 == L:
                out.append(n / 8 + dirs)
            else:
                out.append(n * (rd + wr) + dirs)
        return out
    l = 0
    while l < L:
        rd = in_bytes if l == 0 else mid_bytes
        if l + 1 < L:
            wr = mid_bytes if l + 2 < L else 0
            out.append(n * (rd + wr) + 2 * dirs)
            l += 2
        else:
            out.append(n * rd + dirs)
            l += 1
    assert len(out) == passes, (len(out), passes)
    return out


def traffic_per_launch(workload: str, dominant: bool = False):
    """Measured HBM bytes per level-pass launch from committed rocprofv3
    counter runs (averaged over every level-pass launch, or with `dominant`
    those of the most-launched level-pass kernel), or None when absent or
    taken on different kernel sources."""
    try:
        doc = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    ent = doc.get(workload)
    if not ent or ent.get("source_sha256") != source_sha():
        return None
    if not dominant:
        return ent.get("traffic_bytes_per_launch")
    lp = {k: v for k, v in ent.get("kernels", {}).items() if "level_pass" in k or "pair_pass" in k}
    if not lp:
        return None
    dom = max(lp, key=lambda k: lp[k]["launches"])
    return lp[dom]["fetch_bytes"] + lp[dom]["write_bytes"]


def cpu_info():
    """(model name, online CPUs, CPUs this process may use)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def cpu_baseline(S, sigma, L, sample_n, reps: int = 3):
    """The oracle (sequential, one thread) on the first sample_n symbols:
    bits, C and rank/select, the median of `reps` runs."""
    from oracle import oracle
    sub = S[:sample_n].copy()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        t = oracle.build(sub, sigma)
        oracle.rank_select(t["bits"], t["n"], t["L"])
        times.append(time.perf_counter() - t0)
    dt = sorted(times)[len(times) // 2]
    model, online, avail = cpu_info()
    return {"value": sample_n * L / dt, "unit": "symbols*levels/s", "cores": 1, "kind": "oracle",
            "sample": f"first {sample_n} symbols of the same workload, bits + C + rank/select, single thread "
                      f"(1 of {avail} cores), median of {reps} runs: "
                      + ", ".join(f"{x:.2f}" for x in times) + " s",
            "cpu_model": model, "nproc": avail, "cpus_online": online, "median_of": reps}


PROBE = os.path.join(ROOT, "paper_1407_8142_amd", "bw_probe")


def copy_probe():
    """Achievable streaming rates from the bw_probe executable (a child
    process): grid-stride copy, one 16 KiB tile per block (the level pass's
    pattern) and read-only tiles, in GB/s; None when the probe is missing."""
    import subprocess
    if not os.path.exists(PROBE):
        return None
    try:
        out = subprocess.run([PROBE, "1024", "20"], capture_output=True, text=True, timeout=120, check=True).stdout
    except (subprocess.SubprocessError, OSError):
        return None
    res = {}
    for line in out.splitlines():
        if line.startswith("{"):
            d = json.loads(line)
            res[d["probe"]] = d["GBps"]
    return res or None


def model_bytes(n: int, L: int, b: int) -> float:
    """The levelWT model's algorithmic bytes of one build (one level per
    pass): the histogram read of S, every level's read of its sequence
    (b bytes a symbol) and write of the next (not at the last level), its
    bits, rank entries (1/64 byte a symbol) and select samples left out."""
    return n * b + L * n * (b + 1 / 8) + (L - 1) * n * b + L * n * (1 / 8 + 1 / 64)


def physical_bytes(n: int, L: int, b: int, mid: int) -> float:
    """The bytes the build actually moves with narrowed levels: the sequence
    pass before level 0, then level passes at the narrowed width mid."""
    return n * b + sum(level_pass_bytes(n, L, b, mid, L))


def alphabet_leg(workload: str, steps: int, warmup: int):
    """A large-alphabet workload (n = 2^27 32-bit symbols) built as the tree:
    ms per build, sym*lvl/s, and the HBM rate of the model's bytes and of
    the bytes moved at the narrowed widths."""
    import torch

    from paper_1407_8142_amd import inputs, wt

    desc, n = WORKLOADS[workload]
    log(f"[{workload}] generating n={n}")
    S, sigma = inputs.workload(workload, n)
    L = wt.plan(n, sigma, 4).L
    mid = 1 if L <= 8 else (2 if L <= 16 else 4)
    d = wt.to_device(S)
    del S
    t = wt.WaveletTree.allocate(n, sigma, 4, True, d.device)
    for _ in range(warmup):
        t.build_from(d)
    torch.cuda.synchronize()
    if t.status() != wt.WT_OK:
        raise SystemExit(f"{workload}: input rejected")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        t.build_from(d)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    bm, bp = model_bytes(n, L, 4), physical_bytes(n, L, 4, mid)
    res = {"config": {"workload": desc, "n": n, "sigma": sigma, "levels": L, "sym_bytes": 4,
                      "level_width_bytes": mid, "histogram": wt.histogram_path(n, sigma, 4)},
           "value": n * L / (ms / 1e3), "unit": "symbols*levels/s", "ms_per_step": ms, "steps": steps,
           "model_bytes": bm, "model_GBps": bm / (ms / 1e3) / 1e9,
           "model_frac_of_hbm_peak": bm / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
           "physical_bytes": bp, "physical_GBps": bp / (ms / 1e3) / 1e9,
           "physical_frac_of_hbm_peak": bp / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
    log(f"[{workload}] {ms:.3f} ms/step, {res['value']:.3e} sym*lvl/s, model {res['model_GBps']:.0f} GB/s, "
        f"physical {res['physical_GBps']:.0f} GB/s")
    del t, d
    torch.cuda.empty_cache()
    return res


def batch_model_bytes(jobs) -> float:
    """Algorithmic HBM bytes of one batched build: per job the histogram read
    of S, every level pass (level_pass_bytes) and the C output."""
    total = 0.0
    for n, sigma, b in jobs:
        L = 0 if sigma == 1 else (sigma - 1).bit_length()
        mid = 1 if L <= 8 else (2 if L <= 16 else 4)
        total += n * b + sum(level_pass_bytes(n, L, b, mid, L)) + 8 * (sigma + 1)
    return total


def variant_leg(name: str, build_once, status, n: int, L: int, steps: int, tree_ms: float, launch: str):
    """Times another construction of the same input (after two untimed runs)
    with HIP events, as the tree build is timed; sym*lvl/s counts the binary
    levels (the same information for every variant)."""
    import torch

    from paper_1407_8142_amd import wt

    for _ in range(2):
        build_once()
    torch.cuda.synchronize()
    if status() != wt.WT_OK:
        raise SystemExit(f"input rejected by the {name} build")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        build_once()
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    log(f"[{name}] {ms:.3f} ms/step, {n * L / (ms / 1e3):.3e} sym*lvl/s")
    return {"value": n * L / (ms / 1e3), "unit": "symbols*levels/s", "ms_per_step": ms, "steps": steps,
            "tree_ms_per_step": tree_ms, "launch": launch}


def matrix_leg(d_seq, n: int, sigma: int, sym_bytes: int, L: int, steps: int, tree_ms: float):
    """The same input built as a wavelet matrix (wt_build_matrix, with directories)."""
    from paper_1407_8142_amd import wt

    m = wt.WaveletMatrix.allocate(n, sigma, sym_bytes, True, d_seq.device)
    return variant_leg("matrix", lambda: m.build_from(d_seq), m.status, n, L, steps, tree_ms,
                       "wt_build_matrix on the same input")


def multiary_leg(d_seq, n: int, sigma: int, L: int, steps: int, tree_ms: float):
    """The same byte input built as a 4-ary wavelet tree (wt_build_multiary)."""
    from paper_1407_8142_amd import wt

    t = wt.WaveletMultiary.allocate(n, sigma, d_seq.device)
    return variant_leg("multiary", lambda: t.build_from(d_seq), t.status, n, L, steps, tree_ms,
                       "wt_build_multiary (d = 4, ceil(L/2) levels) on the same input")


def huffman_leg(d_seq, n: int, sigma: int, L: int, steps: int, tree_ms: float):
    """The same byte input built as a Huffman-shaped wavelet tree
    (wt_build_huffman): the step time, the height, the code bits it stores
    (the sum of its level lengths) and their rate beside sym*lvl/s."""
    from paper_1407_8142_amd import wt

    t = wt.WaveletHuffman.allocate(n, sigma, d_seq.device)
    leg = variant_leg("huffman", lambda: t.build_from(d_seq), t.status, n, L, steps, tree_ms,
                      "wt_build_huffman (one wait for the height, then a level pass per level) on the same input")
    bits = int(t.nd[: t.h].sum().item())
    leg.update({"height": t.h, "code_bits": bits, "code_bits_per_symbol": round(bits / max(n, 1), 4),
                "code_bits_per_s": bits / (leg["ms_per_step"] / 1e3)})
    log(f"[huffman] height {t.h}, {bits / max(n, 1):.3f} code bits per symbol, "
        f"{leg['code_bits_per_s']:.3e} code bits/s")
    return leg


def sort_leg(d_seq, n: int, sigma: int, L: int, steps: int, tree_ms: float):
    """The same byte input built by sortWT (wt_build_sort): a sorted copy of S
    per level instead of the level passes, the same outputs."""
    from paper_1407_8142_amd import wt

    t = wt.WaveletTree.allocate(n, sigma, 1, True, d_seq.device)
    wt.build_sort(d_seq, sigma, tree=t)  # grows the scratch once
    return variant_leg("sort", lambda: wt.build_sort(d_seq, sigma, tree=t), t.status, n, L, steps, tree_ms,
                       "wt_build_sort (every level from S stably sorted by its top l bits) on the same input")


def batch_leg(count: int, steps: int, tune=None, per_seq_check: bool = True):
    """Batched build vs one wt_build per sequence, same outputs, same GPU.
    ``tune`` (mode, blocks_per_cu, chunk) skips the autotuner; without the
    per-sequence check only the batched build runs (for profiling it)."""
    import ctypes

    import torch

    from paper_1407_8142_amd import autotune, inputs, wt

    log(f"[batch] generating {count} sequences")
    seqs = inputs.batch(count=count)
    jobs = [(q.S.size, q.sigma, q.S.dtype.itemsize) for q in seqs]
    sym_lvl = sum(n * (0 if s == 1 else (s - 1).bit_length()) for n, s, _ in jobs)
    dev = [wt.to_device(q.S) for q in seqs]
    b = wt.Batch(dev, [q.sigma for q in seqs])
    b.slab.fill_(-1)  # padding between buffers is never written: keep it equal in both runs
    log(f"[batch] {b.layout.items} work items, scratch {b.layout.scratch_bytes / 2**30:.2f} GiB, "
        f"outputs {b.slab.numel() * 8 / 2**30:.2f} GiB; autotuning")
    if tune is None:
        best, table, fused = autotune.autotune(b)
    else:
        fused = tune[3] if len(tune) > 3 else 1
        best, table = wt.Tune(mode=tune[0], blocks_per_cu=tune[1], chunk=tune[2], spin_limit=0), []
        wt.set_fused_levels(fused)
    log(f"[batch] best tune {best.as_dict()} fused={fused}: " + ", ".join(
        f"{r['tune']['mode']}/{r['tune']['blocks_per_cu']}/{r['tune']['chunk']}/f{int(r['fused'])}={r['ms']}"
        for r in table))
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        b.run(best, stream=stream)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=stream):
            b.run(best, stream=stream)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    rc, codes = b.status()
    if rc != wt.WT_OK:
        raise SystemExit(f"batched build failed: {wt.STATUS_NAMES.get(rc, rc)}")
    cur = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(cur)
    for _ in range(steps):
        g.replay()
    e1.record(cur)
    torch.cuda.synchronize()
    batch_ms = e0.elapsed_time(e1) / steps
    wt.set_fused_levels(1)  # the captured graph keeps the tuned setting; later builds take the default
    model = batch_model_bytes(jobs)
    if not per_seq_check:
        log(f"[batch] batched {batch_ms:.3f} ms ({best.as_dict()})")
        return {"ms_per_step": batch_ms, "value": sym_lvl / (batch_ms / 1e3), "unit": "symbols*levels/s",
                "tune": best.as_dict(), "fused_tail_levels": fused, "model_bytes": model,
                "model_frac_of_hbm_peak": model / (batch_ms / 1e3) / 1e9 / HBM_PEAK_GBS}
    want = b.slab.clone()

    # One wt_build per sequence into the same output buffers, one scratch
    # buffer reused in stream order.
    lib = wt.lib()
    scratch_bytes = max(wt.plan(n, s, w).scratch_bytes for n, s, w in jobs)
    scratch = torch.empty(scratch_bytes, dtype=torch.uint8, device="cuda")
    outs = [t.outputs() for t in b.trees]
    args = [(wt._ptr(q), n, s, w) for q, (n, s, w) in zip(dev, jobs)]
    sp, sbytes = wt._ptr(scratch), scratch.numel()

    def per_seq(stream_handle):
        for (p, n, s, w), o in zip(args, outs):
            rc = lib.wt_build(p, n, s, w, ctypes.byref(o), sp, sbytes, stream_handle)
            if rc:
                raise SystemExit(f"wt_build failed: {rc}")

    per_seq(cur.cuda_stream)  # warm-up
    torch.cuda.synchronize()
    b.slab.fill_(-1)
    torch.cuda.synchronize()
    reps = max(1, min(steps, 3))
    w0 = time.perf_counter()
    e0.record(cur)
    for _ in range(reps):
        per_seq(cur.cuda_stream)
    e1.record(cur)
    torch.cuda.synchronize()
    per_seq_ms = e0.elapsed_time(e1) / reps
    per_seq_wall_ms = (time.perf_counter() - w0) * 1e3 / reps
    identical = bool(torch.equal(b.slab, want))
    log(f"[batch] batched {batch_ms:.3f} ms, per-sequence {per_seq_ms:.3f} ms (wall {per_seq_wall_ms:.3f}), "
        f"identical={identical}")
    return {
        "config": {"workload": f"batched build: {count} sequences, lengths log-uniform in [2^10, 2^20], "
                               "sigma uniform over {4, 256, 2^16} (u8/u8/u16), uniform symbols",
                   "sequences": count, "symbols": sum(n for n, _, _ in jobs), "symbols_levels": sym_lvl},
        "value": sym_lvl / (batch_ms / 1e3), "unit": "symbols*levels/s", "ms_per_step": batch_ms,
        "steps": steps, "launch": "wt_batch_run captured in one graph (" + (
            "one persistent work-queue launch" if best.mode == wt.BATCH_PERSISTENT else "one launch per phase")
        + " + a clearing kernel)", "tune": best.as_dict(), "fused_tail_levels": fused, "autotune": table,
        "per_seq": {"value": sym_lvl / (per_seq_ms / 1e3), "ms_per_step": per_seq_ms,
                    "wall_ms_per_step": per_seq_wall_ms, "launch": "one wt_build per sequence on one stream"},
        "speedup_vs_per_seq": per_seq_ms / batch_ms, "bit_exact_vs_per_seq": identical,
        "model_bytes": model, "model_gbs": model / (batch_ms / 1e3) / 1e9,
        "model_frac_of_hbm_peak": model / (batch_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
    }


def serve_leg(seconds: float, budget_gb: float, pool: int, h2d_seconds: float, h2d_pool: int):
    """Serving loop on a Poisson trace.  Payloads come from a pool of
    distinct requests (request i carries payload i % pool) staged in HBM
    before the trace; a second, shorter trace takes them from pinned host
    memory instead, so the host-to-device copy is part of every latency."""
    import torch

    from paper_1407_8142_amd import inputs, serve

    def one(sec, index, pool_size, h2d=False, max_requests=None):
        reqs, qtimes = inputs.serving_arrivals(sec, index=index, max_requests=max_requests, pool=pool_size)
        P = min(pool_size, len(reqs))
        log(f"[serve] {len(reqs)} requests over a pool of {P} payloads "
            f"({sum(r.n for r in reqs[:P]) / 1e9:.2f} G symbols staged), {len(qtimes)} query batches"
            + (", payloads in pinned host memory" if h2d else ""))
        slab, layout0, views0 = inputs.stage_requests(reqs[:P])
        host = None
        if h2d:
            host, hviews = inputs.stage_pinned(slab, reqs[:P], layout0)
            payloads = [hviews[i % P] for i in range(len(reqs))]
        else:
            payloads = [views0[i % P] for i in range(len(reqs))]
        layout = [layout0[i % P] for i in range(len(reqs))]
        torch.cuda.synchronize()
        srv = serve.Server(budget_bytes=int(budget_gb * 2**30))
        t0 = time.perf_counter()
        stats = serve.run_trace(srv, reqs, payloads, qtimes, slab, layout, qsize=100_000, seed=index)
        elapsed = time.perf_counter() - t0
        out = serve.summary(stats, elapsed)
        out["requests"] = len(reqs)
        out["payload_pool"] = P
        out["offered_symbols_levels"] = sum(r.n * (0 if r.sigma == 1 else (r.sigma - 1).bit_length()) for r in reqs)
        out["budget_gb"] = budget_gb
        out["streams"] = {"single_builds": len(srv.streams), "batched_builds": 1, "queries": 1}
        log(f"[serve] {out['builds']} builds in {elapsed:.2f} s, {out['evictions']} evictions, build p50/p99 "
            f"{out['build_latency_ms']['p50']}/{out['build_latency_ms']['p99']} ms, query batch p50/p99 "
            f"{out['query_batch_latency_ms']['p50']}/{out['query_batch_latency_ms']['p99']} ms")
        del srv, slab, views0, payloads, host
        torch.cuda.empty_cache()
        return out

    one(0.05, 1, 60, max_requests=60)  # warm-up: kernel loading, allocator growth
    res = one(seconds, 0, pool)
    res["h2d_included"] = one(h2d_seconds, 2, h2d_pool, h2d=True)
    res["config"] = {"workload": "serving: Poisson build requests at 2000/s, n log-uniform in [2^12, 2^26], sigma "
                                 "log-uniform in [2^2, 2^20], Zipf(1.1) symbols permuted; Poisson query batches at "
                                 "100/s of 10^5 queries (half access, half rank with c = S[j]) over the resident "
                                 f"trees; {budget_gb:g} GB resident budget, LRU eviction",
                     "trace_seconds": seconds, "h2d": "excluded: payloads staged in HBM before their arrival "
                                                      "(the h2d_included object copies them from pinned host "
                                                      "memory after admission)"}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # About 0.1 s of builds at the default workload: the GPU's clocks are
    # still rising during the first tens of milliseconds of load.
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="text256", choices=sorted(WORKLOADS))
    ap.add_argument("--n", type=int, default=None, help="override the sequence length")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 27)
    ap.add_argument("--no-matrix", action="store_true",
                    help="skip the wavelet-matrix, 4-ary, Huffman-shaped and sortWT builds of the same input")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-build comparison")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched build (no per-sequence comparison) and print its object")
    ap.add_argument("--batch-tune", default=None, help="MODE,BLOCKS_PER_CU,CHUNK[,FUSED_LEVELS] instead of autotuning "
                    "(fused levels as wt_set_fused_levels takes them; default 1)")
    ap.add_argument("--no-alphabets", action="store_true",
                    help="skip the large-alphabet builds (n = 2^27 32-bit symbols, sigma 2^16 and 2^20)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving trace")
    ap.add_argument("--serve-seconds", type=float, default=6.0)
    ap.add_argument("--serve-budget-gb", type=float, default=16.0)
    ap.add_argument("--serve-pool", type=int, default=1000, help="distinct payloads the trace cycles over")
    ap.add_argument("--serve-h2d-seconds", type=float, default=1.5)
    ap.add_argument("--serve-h2d-pool", type=int, default=300)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1407_8142_amd import inputs, wt

    batch_tune = tuple(int(x) for x in args.batch_tune.split(",")) if args.batch_tune else None
    if args.batch_only:
        print(json.dumps(batch_leg(args.batch_count, args.batch_steps, batch_tune, per_seq_check=False)), flush=True)
        return
    desc, n_default = WORKLOADS[args.workload]
    n = args.n or n_default
    log(f"[bench] generating {args.workload} n={n}")
    S, sigma = inputs.workload(args.workload, n)
    L = wt.plan(n, sigma, S.dtype.itemsize).L
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d_seq = wt.to_device(S, dev)
    tree = wt.WaveletTree.allocate(n, sigma, S.dtype.itemsize, True, dev)
    stream = torch.cuda.current_stream()

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        tree.build_from(d_seq)
    torch.cuda.synchronize()
    if tree.status() != wt.WT_OK:
        raise SystemExit("input rejected by wt_build")
    wt.timing_collect()

    # The level-pass launch times: K builds in which every level-pass launch
    # carries a start and a stop HIP event in its own dispatch
    # (hipExtLaunchKernel, on the launch stream), so the events time the
    # kernel itself.  The step time comes from the K builds after them.
    log(f"[bench] timing the level-pass launches of {args.steps} steps")
    wt.timing_enable(True)
    ev2, ev3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev2.record(stream)
    for _ in range(args.steps):
        tree.build_from(d_seq)
    ev3.record(stream)
    torch.cuda.synchronize()
    wt.timing_enable(False)
    launches = wt.timing_collect()
    ms_per_step_timed = ev2.elapsed_time(ev3) / args.steps
    log(f"[bench] {ms_per_step_timed:.3f} ms/step with per-launch events")

    # The step time: K builds back to back, bracketed by two events.
    log(f"[bench] timing {args.steps} steps")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        tree.build_from(d_seq)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_total = ev0.elapsed_time(ev1)
    ms_per_step = ms_total / args.steps
    value = n * L * args.steps / (ms_total / 1e3)
    log(f"[bench] {ms_per_step:.3f} ms/step (wall {wall / args.steps * 1e3:.3f} ms/step), {value:.3e} sym*lvl/s")

    mid = 1 if L <= 8 else (2 if L <= 16 else 4)
    passes = len(launches) // args.steps
    assert passes * args.steps == len(launches) and passes in (L, (L + 1) // 2), (len(launches), L, args.steps)
    # Byte alphabets without a histogram pass: level L-2 writes the last
    # level's bits, and the last launch is a directory pass over them.
    lastbits = passes == L and L >= 2 and wt.histogram_path(n, sigma, S.dtype.itemsize) == wt.HIST_LEVELS
    per_pass = level_pass_bytes(n, L, S.dtype.itemsize, mid, passes, lastbits)
    per_pass_ms = [sum(launches[i::passes]) / args.steps for i in range(passes)]
    # The dominant kernel: the level passes.  For byte alphabets that is the
    # pass of levels 0..L-3; level L-2's pass (which also writes the last
    # level's bits, and no sequence) and the last level's directory pass are
    # other kernels, reported beside it.
    npass = passes - 2 if lastbits and passes >= 3 else (passes - 1 if lastbits else passes)
    lp_ms = sum(per_pass_ms[:npass]) * args.steps
    lp_bytes = sum(per_pass[:npass]) * args.steps
    avg_launch_ms = lp_ms / (npass * args.steps)
    avg_bytes = lp_bytes / (npass * args.steps)
    achieved = avg_bytes / (avg_launch_ms / 1e3) / 1e9
    log(f"[bench] {'levels per pass: 1' if passes == L else 'levels per pass: 2'}; ms per pass: "
        + " ".join(f"{x:.4f}" for x in per_pass_ms))
    traffic = traffic_per_launch(args.workload if n == n_default else "", dominant=lastbits and passes >= 3)
    probe = copy_probe()
    step_bytes = model_bytes(n, L, S.dtype.itemsize)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "achievable": probe, "frac_of_tile_copy": round(achieved / probe["copy_tile"], 4) if probe else None,
            "step_model_bytes": step_bytes,
            "step_frac": round(step_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "kernel": ("level_pass_u8 (levels 0..L-3)" if lastbits and passes >= 3
                       else "level_pass (all levels)") if passes == L else
                      "pair_pass (two levels per launch; an odd last level by level_pass)",
            "passes_per_build": passes, "avg_launch_ms": round(avg_launch_ms, 5),
            "algorithmic_bytes_per_launch": round(avg_bytes), "level_pass_share_of_step":
                round(lp_ms / args.steps / ms_per_step_timed, 3),
            "ms_per_launch": [round(x, 5) for x in per_pass_ms],
            "level_L_minus_2": ({"kernel": "level_pass_u8 of level L-2 (also writes the last level's bits, "
                                           "no sequence)", "ms": round(per_pass_ms[-2], 5), "bytes": per_pass[-2],
                                 "GBps": round(per_pass[-2] / (per_pass_ms[-2] / 1e3) / 1e9, 1)}
                                if lastbits and passes >= 3 else None),
            "last_level": ({"kernel": "level_dirs (directories over the last level's bits)",
                            "ms": round(per_pass_ms[-1], 5), "bytes": per_pass[-1]} if lastbits else None),
            "launch_timing": "K steps before the timed ones, each level-pass launch carrying its start and "
                             f"stop events in its dispatch ({ms_per_step_timed:.3f} ms/step there)"}

    cpu = None
    if not args.no_cpu_baseline:
        sample = min(args.cpu_sample, n)
        log(f"[bench] cpu baseline: oracle on {sample} symbols")
        cpu = cpu_baseline(S, sigma, L, sample)

    matrix = None if args.no_matrix else matrix_leg(d_seq, n, sigma, S.dtype.itemsize, L, args.steps, ms_per_step)
    multiary = None if args.no_matrix or S.dtype.itemsize != 1 else multiary_leg(d_seq, n, sigma, L, args.steps,
                                                                                ms_per_step)
    huffman = None if args.no_matrix or S.dtype.itemsize != 1 or sigma > 256 else huffman_leg(
        d_seq, n, sigma, L, args.steps, ms_per_step)
    sortwt = None if args.no_matrix or S.dtype.itemsize != 1 or sigma > 256 else sort_leg(
        d_seq, n, sigma, L, args.steps, ms_per_step)
    alphabets = None
    if not args.no_alphabets and args.workload == "text256":
        alphabets = {w: alphabet_leg(w, 10, 10) for w in ("alpha16", "alpha20")}
    batch = None if args.no_batch else batch_leg(args.batch_count, args.batch_steps, batch_tune)
    served = None if args.no_serve else serve_leg(args.serve_seconds, args.serve_budget_gb, args.serve_pool,
                                                  args.serve_h2d_seconds, args.serve_h2d_pool)

    line = {
        "metric": METRIC, "value": value, "unit": "symbols*levels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {1: "u8", 2: "u16", 4: "u32"}[S.dtype.itemsize], "data": "synthetic",
        "config": {"workload": desc if n == n_default else f"{desc} (n overridden to {n})", "n": n,
                   "sigma": sigma, "levels": L, "sym_bytes": S.dtype.itemsize, "directories": True,
                   "input_sha256": inputs.sha256(S)[:16]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "matrix": matrix,
        "multiary": multiary,
        "huffman": huffman,
        "sort": sortwt,
        "alphabets": alphabets,
        "batch": batch,
        "serve": served,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
