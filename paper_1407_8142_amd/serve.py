"""Serving: build wavelet trees as requests arrive, keep the finished trees
resident in HBM, and answer batches of access/rank/select queries on them.

Scheduling (one host thread; every step of construction and every query
runs in the library's kernels):
  admission   requests wait in arrival order; the head is admitted when its
              HBM footprint (outputs + build scratch) fits the budget next
              to what is resident or in flight, after evicting least
              recently used trees that no in-flight query batch is reading
  continuous  each scheduler tick takes every admitted request: the small
  batching    ones (n and sigma under thresholds) go to one batched build
              (wt_batch_run, one launch per phase), each large one to
              wt_build on the next of several streams, so builds that
              arrive while others run overlap with them on the device
  queries     a query batch names trees resident when it arrives; they are
              pinned (not evicted) until its single wt_query_multi launch
              completes
Latency is arrival -> completion as seen by the host loop (polling HIP
events).  A request's payload is either a device tensor (staged in HBM by
the client before its arrival: no host-to-device transfer in the latency)
or a pinned host tensor, copied to the device on the build's stream after
admission (the transfer is part of the latency and of the footprint).

Streams: two for single builds, one for batched builds, one for query
batches (the device's four hardware queues), plus a copy-only stream for
the batches' job tables and one for status reads.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import wt


@dataclass
class BuildRequest:
    rid: int
    seq: torch.Tensor  # symbols (1-, 2- or 4-byte): a device tensor, 16-byte aligned, or a pinned host tensor
    sigma: int
    arrival: float     # seconds on the server clock


@dataclass
class QueryBatch:
    qid: int
    arrival: float
    targets: list          # request ids of the trees the batch reads
    tree: torch.Tensor     # int32 index into targets, per query (device)
    kind: torch.Tensor     # uint8 wt.Q_* per query (device)
    a: torch.Tensor        # int64 (device)
    b: torch.Tensor        # int64 (device)


@dataclass
class _Resident:
    tree: "wt.WaveletTree"
    nbytes: int
    owner: object          # the allocation the tree's buffers live in (freed with its last tree)
    pins: int = 0
    sym_levels: int = 0


@dataclass
class _InflightBuild:
    reqs: list
    event: torch.cuda.Event
    trees: list
    nbytes: list
    owner: object
    batch: "wt.Batch | None" = None
    status_host: torch.Tensor | None = None
    scratch_bytes: int = 0   # build scratch and device copies of host payloads, freed when it completes
    payloads: list = field(default_factory=list)


@dataclass
class Stats:
    build_latency: list = field(default_factory=list)
    query_latency: list = field(default_factory=list)
    built: int = 0
    sym_levels: int = 0
    queries: int = 0
    evictions: int = 0
    batches: int = 0
    singles: int = 0
    failed: list = field(default_factory=list)


def _levels(sigma: int) -> int:
    return 0 if sigma <= 1 else (sigma - 1).bit_length()


class _Slab:
    """The trees of one batched build share one allocation: it stays
    charged to the budget, whole, until its last tree is gone."""

    def __init__(self, tensors, nbytes: int, members: int):
        self.tensors = tensors
        self.nbytes = nbytes
        self.live = members


class Server:
    def __init__(self, budget_bytes: int, build_streams: int = 2, small_n: int = 1 << 20, small_sigma: int = 1 << 14,
                 max_batch: int = 1024, tune: "wt.Tune | None" = None, clock=time.perf_counter):
        self.budget = int(budget_bytes)
        self.small_n, self.small_sigma, self.max_batch = small_n, small_sigma, max_batch
        self.tune = tune if tune is not None else wt.Tune(mode=wt.BATCH_PER_PHASE)
        self.streams = [torch.cuda.Stream() for _ in range(max(1, build_streams))]
        self.batch_stream = torch.cuda.Stream()
        self.upload_stream = torch.cuda.Stream()
        self.query_stream = torch.cuda.Stream()
        self.status_stream = torch.cuda.Stream()  # idle: status reads never wait on queued builds
        self._next_stream = 0
        self.pending: collections.deque = collections.deque()
        self.inflight: list[_InflightBuild] = []
        self.resident: "collections.OrderedDict[int, _Resident]" = collections.OrderedDict()
        self.queries_inflight: list = []
        self.in_use = 0  # bytes resident + in flight
        self.stats = Stats()
        self.clock = clock
        self.t0 = clock()
        self.results: dict[int, torch.Tensor] = {}
        self.keep_results = False

    # -- client side -------------------------------------------------------
    def now(self) -> float:
        return self.clock() - self.t0

    def submit_build(self, req: BuildRequest):
        self.pending.append(req)

    def submit_queries(self, qb: QueryBatch):
        trees = []
        for rid in qb.targets:
            r = self.resident.get(rid)
            if r is None:
                raise KeyError(f"tree {rid} is not resident")
            r.pins += 1
            self.resident.move_to_end(rid)
            trees.append(r.tree)
        s = self.query_stream
        with torch.cuda.stream(s):
            views = wt.views_tensor(trees)
            out = wt.query_multi(views, len(trees), qb.tree, qb.kind, qb.a, qb.b, stream=s)
        ev = torch.cuda.Event()
        ev.record(s)
        self.queries_inflight.append((qb, ev, out, views))

    def resident_ids(self) -> list[int]:
        return list(self.resident.keys())

    def tree(self, rid: int) -> "wt.WaveletTree":
        return self.resident[rid].tree

    # -- accounting ----------------------------------------------------------
    @staticmethod
    def footprint(n: int, sigma: int, sym_bytes: int) -> tuple[int, int]:
        """(output bytes, build scratch bytes) of one tree."""
        lay, shapes = wt.WaveletTree.output_words(n, sigma, sym_bytes)
        out = 0
        for sh in shapes:
            w = 1
            for d in sh:
                w *= d
            out += 8 * (-(-w // 32) * 32)
        return out, int(lay.scratch_bytes)

    def _release(self, owner, nbytes: int):
        """A tree is gone: its own bytes, or its slab's once the slab's last
        tree is gone."""
        if isinstance(owner, _Slab):
            owner.live -= 1
            if owner.live == 0:
                owner.tensors = None
                self.in_use -= owner.nbytes
        else:
            self.in_use -= nbytes

    def _evict_for(self, need: int) -> bool:
        for rid in list(self.resident.keys()):
            if self.in_use + need <= self.budget:
                break
            r = self.resident[rid]
            if r.pins:
                continue
            del self.resident[rid]
            self._release(r.owner, r.nbytes)
            self.stats.evictions += 1
        return self.in_use + need <= self.budget

    # -- scheduler -----------------------------------------------------------
    def _admit(self) -> tuple[list, list]:
        small, large = [], []
        while self.pending:
            req = self.pending[0]
            n, sb = req.seq.numel(), req.seq.element_size()
            out_b, scr_b = self.footprint(n, req.sigma, sb)
            if not req.seq.is_cuda:
                scr_b += -(-(n * sb) // 256) * 256  # the device copy of the payload
            need = out_b + scr_b
            if need > self.budget:
                self.pending.popleft()
                self.stats.failed.append((req.rid, "larger than the budget"))
                continue
            if self.in_use + need > self.budget and not self._evict_for(need):
                break
            self.pending.popleft()
            self.in_use += need
            if n <= self.small_n and req.sigma <= self.small_sigma and len(small) < self.max_batch:
                small.append((req, out_b, scr_b))
            else:
                large.append((req, out_b, scr_b))
        return small, large

    @staticmethod
    def _on_device(seq: torch.Tensor, stream) -> torch.Tensor:
        """The payload on the device: itself, or its copy made on `stream`."""
        if seq.is_cuda:
            return seq
        with torch.cuda.stream(stream):
            return seq.to("cuda", non_blocking=True)

    def _launch_large(self, req, out_b, scr_b):
        s = self.streams[self._next_stream]
        self._next_stream = (self._next_stream + 1) % len(self.streams)
        n, sb = req.seq.numel(), req.seq.element_size()
        seq = self._on_device(req.seq, s)
        with torch.cuda.stream(s):
            t = wt.WaveletTree.allocate(n, req.sigma, sb, True, seq.device)
            t.build_from(seq, stream=s)
            st = torch.empty(1, dtype=torch.int32, pin_memory=True)
            st.copy_(t.scratch[:4].view(torch.int32), non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(s)
        self.inflight.append(_InflightBuild([req], ev, [t], [out_b], None, None, st, scr_b, [seq]))
        self.stats.singles += 1

    def _launch_small(self, group):
        reqs = [g[0] for g in group]
        s = self.batch_stream
        # Host payloads are copied on the batch stream, ahead of the batch's
        # launches there (its job tables, on the upload stream, hold only
        # their addresses).
        seqs = [self._on_device(r.seq, s) for r in reqs]
        b = wt.Batch(seqs, [r.sigma for r in reqs], stream=self.upload_stream)
        with torch.cuda.stream(s):
            b.run(self.tune, stream=s)
        ev = torch.cuda.Event()
        ev.record(s)
        # Outputs of the whole group share one slab (charged whole until its
        # last tree goes); the group's scratch estimate is replaced by the
        # batch's own scratch plus its payload copies.
        copies = sum(-(-(q.numel() * q.element_size()) // 256) * 256 for r, q in zip(reqs, seqs)
                     if not r.seq.is_cuda)
        scr = int(b.layout.scratch_bytes) + copies
        est_scr = sum(g[2] for g in group)
        self.in_use += scr - est_scr
        est_out = sum(g[1] for g in group)
        self.inflight.append(_InflightBuild(reqs, ev, b.trees, [g[1] for g in group],
                                            _Slab([b.slab], est_out, len(reqs)), b, None, scr, seqs))
        self.stats.batches += 1

    def _retire(self) -> bool:
        progress = False
        keep = []
        for f in self.inflight:
            if not f.event.query():
                keep.append(f)
                continue
            progress = True
            done = self.now()
            if f.batch is not None:
                rc, codes = f.batch.status(stream=self.status_stream)
                f.batch.scratch = None
            else:
                codes = [wt.WT_OK if int(f.status_host[0]) == 0 else wt.WT_ERR_SYMBOL]
                # drop the scratch (a slice would keep its storage alive)
                f.trees[0].scratch = torch.empty(0, dtype=torch.uint8, device=f.trees[0].scratch.device)
            self.in_use -= f.scratch_bytes
            f.payloads = []
            for req, t, nb, code in zip(f.reqs, f.trees, f.nbytes, codes):
                if code != wt.WT_OK:
                    self.stats.failed.append((req.rid, wt.STATUS_NAMES.get(code, code)))
                    self._release(f.owner, nb)
                    continue
                sl = t.n * t.L
                self.resident[req.rid] = _Resident(t, nb, f.owner, 0, sl)
                self.stats.build_latency.append(done - req.arrival)
                self.stats.built += 1
                self.stats.sym_levels += sl
        self.inflight = keep
        qkeep = []
        for qb, ev, out, views in self.queries_inflight:
            if not ev.query():
                qkeep.append((qb, ev, out, views))
                continue
            progress = True
            self.stats.query_latency.append(self.now() - qb.arrival)
            self.stats.queries += int(qb.tree.numel())
            for rid in qb.targets:
                r = self.resident.get(rid)
                if r is not None:
                    r.pins -= 1
            if self.keep_results:
                self.results[qb.qid] = out
        self.queries_inflight = qkeep
        return progress

    def pump(self) -> bool:
        """One scheduler tick; True if anything changed."""
        progress = self._retire()
        small, large = self._admit()
        for req, out_b, scr_b in large:
            self._launch_large(req, out_b, scr_b)
        if small:
            self._launch_small(small)
        return progress or bool(small) or bool(large)

    def idle(self) -> bool:
        return not self.pending and not self.inflight and not self.queries_inflight

    def drain(self, timeout_s: float = 120.0):
        end = self.clock() + timeout_s
        while not self.idle():
            if self.clock() > end:
                raise TimeoutError("server did not drain")
            if not self.pump():
                time.sleep(50e-6)


def percentile(xs, q):
    if not xs:
        return None
    return float(np.percentile(np.asarray(xs), q))


def make_query_batch(qid: int, arrival: float, ids: list, sizes: dict, slab: torch.Tensor, layout: dict,
                     qsize: int, gen: torch.Generator, select_share: float = 0.0) -> QueryBatch:
    """Client side: `qsize` queries over the trees `ids` (uniformly), half
    access(i) with i uniform in [0, n), half rank(c, i) with c = S[j] for a
    uniform j and i uniform in [0, n] (a `select_share` of the rank queries
    become select(c, k) with k uniform in [1, 8]).  S[j] is read from the
    staged payload slab."""
    dev = slab.device
    k = len(ids)
    n_t = torch.tensor([sizes[r] for r in ids], dtype=torch.float64, device=dev)
    off_t = torch.tensor([layout[r][0] for r in ids], dtype=torch.int64, device=dev)
    w_t = torch.tensor([layout[r][1] for r in ids], dtype=torch.int64, device=dev)
    tree = torch.randint(0, k, (qsize,), generator=gen, device=dev, dtype=torch.int64)
    nq = n_t[tree]
    u = torch.rand(4, qsize, generator=gen, device=dev, dtype=torch.float64)
    is_access = u[0] < 0.5
    i_acc = torch.floor(u[1] * nq).to(torch.int64)
    j = torch.minimum(torch.floor(u[2] * nq), nq - 1).to(torch.int64)
    i_rank = torch.floor(u[3] * (nq + 1)).to(torch.int64)
    wq, base = w_t[tree], off_t[tree] + j * w_t[tree]
    c = slab[base].to(torch.int64)
    last = slab.numel() - 1
    for byte in (1, 2, 3):  # little-endian symbol bytes beyond the first
        hi = slab[torch.clamp(base + byte, max=last)].to(torch.int64) << (8 * byte)
        c = c + torch.where(wq > byte, hi, torch.zeros_like(c))
    kind = torch.where(is_access, torch.full_like(tree, wt.Q_ACCESS), torch.full_like(tree, wt.Q_RANK))
    a = torch.where(is_access, i_acc, c)
    b = torch.where(is_access, torch.zeros_like(i_acc), i_rank)
    if select_share > 0:
        sel = (~is_access) & (torch.rand(qsize, generator=gen, device=dev, dtype=torch.float64) < select_share)
        kind = torch.where(sel, torch.full_like(kind, wt.Q_SELECT), kind)
        b = torch.where(sel, torch.randint(1, 9, (qsize,), generator=gen, device=dev, dtype=torch.int64), b)
    return QueryBatch(qid, arrival, list(ids), tree.to(torch.int32), kind.to(torch.uint8), a, b)


def run_trace(server: Server, reqs: list, views: list, qtimes: list, slab: torch.Tensor, layout: list,
              qsize: int = 100_000, seed: int = 0, select_share: float = 0.0, timeout_s: float = 300.0):
    """Replays the trace in real time: request r arrives at reqs[r].arrival_s
    (payload views[r]), query batch q at qtimes[q] over the trees resident
    then.  Returns the server's Stats."""
    sizes = {r: req.n for r, req in enumerate(reqs)}
    lay = {r: layout[r] for r in range(len(reqs))}
    gen = torch.Generator(device=slab.device)
    gen.manual_seed(seed)
    torch.cuda.synchronize()
    server.t0 = server.clock()
    i = qi = 0
    end = server.clock() + timeout_s
    while i < len(reqs) or qi < len(qtimes) or not server.idle():
        if server.clock() > end:
            raise TimeoutError("trace did not finish")
        now = server.now()
        while i < len(reqs) and reqs[i].arrival_s <= now:
            server.submit_build(BuildRequest(i, views[i], reqs[i].sigma, reqs[i].arrival_s))
            i += 1
        while qi < len(qtimes) and qtimes[qi] <= now:
            ids = server.resident_ids()
            if ids:
                server.submit_queries(make_query_batch(qi, qtimes[qi], ids, sizes, slab, lay, qsize, gen,
                                                       select_share))
            qi += 1
        if not server.pump():
            time.sleep(20e-6)
    return server.stats


def summary(stats: Stats, elapsed_s: float) -> dict:
    return {
        "builds": stats.built, "failed": len(stats.failed), "evictions": stats.evictions,
        "batched_launches": stats.batches, "single_builds": stats.singles,
        "build_latency_ms": {"p50": _ms(percentile(stats.build_latency, 50)),
                             "p99": _ms(percentile(stats.build_latency, 99))},
        "query_batch_latency_ms": {"p50": _ms(percentile(stats.query_latency, 50)),
                                   "p99": _ms(percentile(stats.query_latency, 99))},
        "builds_per_s": stats.built / elapsed_s, "symbols_levels_per_s": stats.sym_levels / elapsed_s,
        "queries_per_s": stats.queries / elapsed_s, "query_batches": len(stats.query_latency),
        "elapsed_s": elapsed_s,
    }


def _ms(x):
    return None if x is None else round(x * 1e3, 3)
