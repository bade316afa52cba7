"""Seeded synthetic workloads.

This module only draws random symbols; it holds none of the wavelet-tree
arithmetic.  It serves the tests, the smoke check and the benchmark alike.

Workloads (the paper's real corpora are not available; these stand in for the
shapes of its inputs -- text with alphabets up to 256, random inputs with
sigma = 2^k, and a document-id array with a large alphabet):

  1  uniform:       n = 2^20 uint8, sigma = 256, i.i.d. uniform
  2  text-like:     n = 2^28 uint8, sigma = 256; runs whose symbol follows
                    Zipf(1.1) over a seeded permutation of the byte alphabet
                    and whose length is geometric with mean 4
  3  large-alpha:   n = 2^27 uint32, sigma in {2^16, 2^20}; the first half
                    uniform, the second half Zipf(1.0) over a seeded
                    permutation of [0, sigma) (concatenated in one input)
  4  batch:         4096 sequences, n = floor(2^U), U ~ U[10, 20], sigma drawn
                    from {4, 256, 2^16} (uint8, uint8, uint16), uniform symbols
  5  serving:       Poisson arrivals (mean gap 0.5 ms), n = floor(2^U) with
                    U ~ U[12, 26], sigma = floor(2^U) with U ~ U[2, 20],
                    narrowest symbol width, Zipf(1.1) symbols over a seeded
                    permutation of [0, sigma)

Seeds are 1407 * 1000 + workload id (plus a sequence index for 4 and 5).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

SEED_BASE = 1407 * 1000


def rng_for(workload: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + workload + index))


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).view(np.uint8)).hexdigest()


def dtype_for_sigma(sigma: int):
    if sigma <= 1 << 8:
        return np.uint8
    if sigma <= 1 << 16:
        return np.uint16
    return np.uint32


def zipf_symbols(rng: np.random.Generator, count: int, ranks: int, s: float,
                 perm: np.ndarray, dtype, chunk: int = 1 << 24) -> np.ndarray:
    """``count`` draws from a truncated Zipf(s) over ``ranks`` ranks (P(r) ~ r^-s,
    r = 1..ranks), mapped to symbols through ``perm`` (inverse-CDF sampling)."""
    w = np.arange(1, ranks + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    out = np.empty(count, dtype=dtype)
    for lo in range(0, count, chunk):
        hi = min(count, lo + chunk)
        u = rng.random(hi - lo)
        r = np.searchsorted(cdf, u, side="right")
        np.minimum(r, ranks - 1, out=r)
        out[lo:hi] = perm[r]
    return out


def uniform(n: int = 1 << 20, sigma: int = 256, seed_workload: int = 1, index: int = 0,
            dtype=None) -> np.ndarray:
    rng = rng_for(seed_workload, index)
    dt = dtype or dtype_for_sigma(sigma)
    return rng.integers(0, sigma, n, dtype=np.uint64).astype(dt)


def text_like(n: int = 1 << 28, sigma: int = 256, s: float = 1.1, mean_run: float = 4.0,
              index: int = 0) -> np.ndarray:
    """Runs of repeated symbols: symbol ~ Zipf(s) over a permuted alphabet,
    run length ~ Geometric(1/mean_run) (support >= 1)."""
    rng = rng_for(2, index)
    perm = rng.permutation(sigma).astype(np.uint64)
    dt = dtype_for_sigma(sigma)
    out = np.empty(n, dtype=dt)
    filled = 0
    while filled < n:
        runs = max(1024, int((n - filled) / mean_run * 1.05) + 1024)
        runs = min(runs, 1 << 24)
        syms = zipf_symbols(rng, runs, sigma, s, perm, dt)
        lens = rng.geometric(1.0 / mean_run, runs)
        piece = np.repeat(syms, lens)
        take = min(n - filled, piece.shape[0])
        out[filled:filled + take] = piece[:take]
        filled += take
    return out


def large_alphabet(n: int = 1 << 27, sigma: int = 1 << 20, index: int = 0) -> np.ndarray:
    """First half uniform over [0, sigma), second half Zipf(1.0) over a permuted [0, sigma)."""
    rng = rng_for(3, index)
    half = n // 2
    a = rng.integers(0, sigma, half, dtype=np.uint64).astype(np.uint32)
    perm = rng.permutation(sigma).astype(np.uint32)
    b = zipf_symbols(rng, n - half, sigma, 1.0, perm, np.uint32)
    return np.concatenate([a, b])


@dataclass
class BatchSeq:
    S: np.ndarray
    sigma: int


def batch(count: int = 4096, lo_exp: float = 10.0, hi_exp: float = 20.0,
          sigmas=(4, 256, 1 << 16), index: int = 0) -> list[BatchSeq]:
    rng = rng_for(4, index)
    out = []
    for _ in range(count):
        n = int(np.floor(2.0 ** rng.uniform(lo_exp, hi_exp)))
        sigma = int(sigmas[rng.integers(0, len(sigmas))])
        S = rng.integers(0, sigma, n, dtype=np.uint64).astype(dtype_for_sigma(sigma))
        out.append(BatchSeq(S, sigma))
    return out


@dataclass
class Request:
    arrival_s: float
    S: np.ndarray
    sigma: int


def serving_requests(count: int, mean_gap_s: float = 0.5e-3, n_exp=(12.0, 26.0),
                     sigma_exp=(2.0, 20.0), s: float = 1.1, index: int = 0) -> list[Request]:
    rng = rng_for(5, index)
    t = 0.0
    out = []
    for _ in range(count):
        t += float(rng.exponential(mean_gap_s))
        n = int(np.floor(2.0 ** rng.uniform(*n_exp)))
        sigma = max(1, int(np.floor(2.0 ** rng.uniform(*sigma_exp))))
        perm = rng.permutation(sigma).astype(np.uint64)
        S = zipf_symbols(rng, n, sigma, s, perm, dtype_for_sigma(sigma))
        out.append(Request(t, S, sigma))
    return out


def workload(cfg: str, n: int | None = None):
    """(S, sigma) for a named single-build workload; ``n`` overrides the length."""
    if cfg == "uniform256":
        return uniform(n or (1 << 20), 256), 256
    if cfg == "text256":
        return text_like(n or (1 << 28)), 256
    if cfg == "alpha16":
        return large_alphabet(n or (1 << 27), 1 << 16), 1 << 16
    if cfg == "alpha20":
        return large_alphabet(n or (1 << 27), 1 << 20), 1 << 20
    raise KeyError(cfg)


# ---------------------------------------------------------------------------
# Serving trace.  Request payloads are generated on the device (the host
# cannot produce ~10^10 symbols per second of trace), from per-request seeds
# drawn by the host generator: Zipf(s) over sigma ranks by inverse CDF on
# the float64 cumulative table, ranks mapped to symbols by a seeded
# permutation -- the same recipe as zipf_symbols, with torch's generator.
@dataclass
class TraceRequest:
    arrival_s: float
    n: int
    sigma: int
    seed: int


def serving_arrivals(seconds: float, rate: float = 2000.0, qrate: float = 100.0, n_exp=(12.0, 26.0),
                     sigma_exp=(2.0, 20.0), index: int = 0, max_requests: int | None = None,
                     pool: int | None = None):
    """Poisson build arrivals (mean rate/s) with n = floor(2^U(n_exp)) and
    sigma = floor(2^U(sigma_exp)), and Poisson query-batch arrivals.  With
    `pool`, request i carries the payload of request i % pool (the first
    `pool` draws: the same size distribution, payloads staged once)."""
    rng = rng_for(5, index)
    reqs, t = [], 0.0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > seconds or (max_requests is not None and len(reqs) >= max_requests):
            break
        if pool is not None and len(reqs) >= pool:
            src = reqs[len(reqs) % pool]
            reqs.append(TraceRequest(t, src.n, src.sigma, src.seed))
            continue
        n = int(np.floor(2.0 ** rng.uniform(*n_exp)))
        sigma = max(2, int(np.floor(2.0 ** rng.uniform(*sigma_exp))))
        reqs.append(TraceRequest(t, n, sigma, int(rng.integers(0, 2**62))))
    qt, t = [], 0.0
    horizon = reqs[-1].arrival_s if reqs else seconds
    while qrate > 0:
        t += float(rng.exponential(1.0 / qrate))
        if t > horizon:
            break
        qt.append(t)
    return reqs, qt


def zipf_device(n: int, sigma: int, s: float, seed: int, out, device="cuda"):
    """Fill `out` (n symbols of the width of `out`'s dtype, a device tensor)
    with Zipf(s) symbols over sigma ranks, permuted, from `seed`."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    w = torch.arange(1, sigma + 1, dtype=torch.float64, device=device).pow_(-s)
    cdf = torch.cumsum(w, 0)
    cdf /= cdf[-1].clone()
    perm = torch.randperm(sigma, generator=g, device=device)
    step = 1 << 24
    for o in range(0, n, step):
        m = min(step, n - o)
        u = torch.rand(m, dtype=torch.float64, generator=g, device=device)
        r = torch.searchsorted(cdf, u).clamp_(max=sigma - 1)
        v = perm[r]
        esz = out.element_size()
        if esz == 1:
            out[o:o + m] = v.to(torch.uint8).view(out.dtype)
        elif esz == 2:
            out[o:o + m] = v.to(torch.int32).view(torch.int16)[::2].view(out.dtype)
        else:
            out[o:o + m] = v.to(torch.int32).view(out.dtype)


def stage_pinned(slab, reqs, layout):
    """A pinned host copy of a staged slab and per-request host views."""
    import torch
    host = torch.empty(slab.numel(), dtype=torch.uint8, pin_memory=True)
    host.copy_(slab)
    dt = {1: torch.uint8, 2: torch.int16, 4: torch.int32}
    return host, [host[o:o + r.n * w].view(dt[w]) for r, (o, w) in zip(reqs, layout)]


def stage_requests(reqs, s: float = 1.1, device="cuda"):
    """All request payloads in one device slab (each 256-byte aligned).
    Returns (slab, [(offset, width)], [tensor view per request])."""
    import torch
    widths = [int(np.dtype(dtype_for_sigma(r.sigma)).itemsize) for r in reqs]
    offs, total = [], 0
    for r, w in zip(reqs, widths):
        offs.append(total)
        total += -(-(r.n * w) // 256) * 256
    slab = torch.empty(max(total, 256), dtype=torch.uint8, device=device)
    views = []
    for r, w, o in zip(reqs, widths, offs):
        v = slab[o:o + r.n * w].view({1: torch.uint8, 2: torch.int16, 4: torch.int32}[w])
        zipf_device(r.n, r.sigma, s, r.seed, v, device)
        views.append(v)
    return slab, list(zip(offs, widths)), views
