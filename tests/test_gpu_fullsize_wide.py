"""Full-size oracle parity for the large alphabets, at the benchmark's sizes
and launch configuration: every output buffer of wt_build (bits, C, rank,
sel1, sel0, sel_counts) equals the oracle's, bit for bit (integer work:
tolerance zero).

- The large-alphabet workload: n = 2^27 32-bit symbols, sigma = 2^16 and
  sigma = 2^20 (first half uniform, second half Zipf(1.0) over a permuted
  alphabet).
- The alphabet of the paper's largest input (sigma = 528155, the document
  array of its Table 1) at n = 2^26, same recipe.
- The two-phase histogram (more than 16 levels over 32-bit symbols) at
  sizes where wt_build takes it (each case asserts that it does): one and
  five coarse bits, a heavy symbol that overflows the 16-bit LDS counters
  many times, a single group, and a rejected symbol.
"""
import sys

import numpy as np
import pytest

from paper_1407_8142_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("bits", "C", "rank", "sel1", "sel0", "sel_counts")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def wtmod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1407_8142_amd import wt
    wt.lib()
    return wt


def gpu_build_np(wt, S, sigma):
    d = wt.to_device(S)
    t = wt.build(d, sigma)
    torch.cuda.synchronize()
    assert t.status() == wt.WT_OK
    got = t.to_numpy()
    del t, d
    torch.cuda.empty_cache()
    return got


def same(got, want, ctx):
    for k in KEYS:
        g = np.asarray(got[k], dtype=np.uint64).reshape(-1)
        w = np.asarray(want[k], dtype=np.uint64).reshape(-1)
        assert g.shape == w.shape, (ctx, k, g.shape, w.shape)
        bad = np.flatnonzero(g != w)
        assert bad.size == 0, f"{ctx}: {k} differs at {bad.size} of {g.size} entries, first {bad[:5]}"


def check(wt, oracle_mod, S, sigma, ctx, path=None):
    n = int(S.size)
    if path is not None:
        assert wt.histogram_path(n, sigma, S.dtype.itemsize) == path, ctx
    say(f"[fullsize-wide] {ctx}: n={n} sigma={sigma} histogram path "
        f"{wt.histogram_path(n, sigma, S.dtype.itemsize)}: GPU build")
    got = gpu_build_np(wt, S, sigma)
    say(f"[fullsize-wide] {ctx}: oracle")
    want = oracle_mod.build_all(S, sigma)
    same(got, want, ctx)
    say(f"[fullsize-wide] {ctx}: equal")


@pytest.mark.parametrize("cfg", ["alpha16", "alpha20"])
def test_large_alphabet_full_size(wtmod, oracle_mod, cfg):
    S, sigma = inputs.workload(cfg)
    path = wtmod.HIST_TWO_PHASE if cfg == "alpha20" else None
    check(wtmod, oracle_mod, S, sigma, f"{cfg} (n=2^27 u32)", path)


def test_document_array_alphabet(wtmod, oracle_mod):
    # sigma of the paper's document array (Table 1): 20 levels, 9 coarse groups
    # past the last full power of two, most of them empty.
    sigma = 528155
    S = inputs.large_alphabet(1 << 26, sigma)
    check(wtmod, oracle_mod, S, sigma, "sigma=528155", wtmod.HIST_TWO_PHASE)


def zipf_ids(rng, n, sigma, s=1.0):
    ranks = np.minimum(rng.zipf(1.0 + s, n) - 1, sigma - 1).astype(np.int64)
    perm = rng.permutation(sigma)
    return perm[ranks].astype(np.uint32)


TWO_PHASE = [
    ("uniform sigma=2^17 (one coarse bit)", 1 << 17, "uniform"),
    ("Zipf sigma=2^20+3 (21 levels, five coarse bits, most groups empty)", (1 << 20) + 3, "zipf"),
    ("70% one symbol, sigma=2^20 (16-bit counters overflow)", 1 << 20, "heavy"),
    ("one group holds everything, sigma=2^20", 1 << 20, "onegroup"),
]


def make(kind, n, sigma, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.integers(0, sigma, n).astype(np.uint32)
    if kind == "zipf":
        return zipf_ids(rng, n, sigma)
    if kind == "heavy":
        S = rng.integers(0, sigma, n).astype(np.uint32)
        S[rng.random(n) < 0.7] = 777777
        return S
    return ((5 << 16) + rng.integers(0, 100, n)).astype(np.uint32)


@pytest.mark.parametrize("ctx,sigma,kind", TWO_PHASE, ids=[c[2] for c in TWO_PHASE])
def test_two_phase_histogram_taken(wtmod, oracle_mod, ctx, sigma, kind):
    n = (1 << 25) + 4099
    S = make(kind, n, sigma, n ^ sigma)
    check(wtmod, oracle_mod, S, sigma, ctx, wtmod.HIST_TWO_PHASE)


def test_two_phase_rejects_bad_symbol(wtmod):
    n, sigma = (1 << 25) + 9, (1 << 18) + 1
    assert wtmod.histogram_path(n, sigma, 4) == wtmod.HIST_TWO_PHASE
    for pos in (0, 12345, n - 1):
        say(f"[fullsize-wide] bad symbol at {pos}: n={n} sigma={sigma}")
        rng = np.random.default_rng(pos)
        S = rng.integers(0, sigma, n).astype(np.uint32)
        S[pos] = sigma + 5
        t = wtmod.build(wtmod.to_device(S), sigma)
        torch.cuda.synchronize()
        assert t.status() == wtmod.WT_ERR_SYMBOL
        del t
        torch.cuda.empty_cache()
