"""GPU parity of the byte-alphabet build without a histogram pass (the
level passes count, per piece of the next level, what its tables need):
every output buffer (bits, C, rank, sel1, sel0, sel_counts) equals the
oracle's, bit for bit (integer work: tolerance zero).  The cases run with
the fused tail levels switched off, so that small inputs take this path
too, and assert that they do; they cover partial tiles, one-tile inputs,
empty nodes (missing symbols, sigma not a power of two), a single symbol,
two extreme symbols, sorted and Zipf-like text, and the symbol check
(sigma < 256) at the first, a middle and the last position."""
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
    wt.set_fused_levels(False)
    yield wt
    wt.set_fused_levels(True)


def assert_same(got, want, ctx):
    for k in KEYS:
        g = np.asarray(got[k], dtype=np.uint64).reshape(-1)
        w = np.asarray(want[k], dtype=np.uint64).reshape(-1)
        assert g.shape == w.shape, (ctx, k, g.shape, w.shape)
        if not np.array_equal(g, w):
            bad = np.flatnonzero(g != w)
            raise AssertionError(f"{ctx}: {k} differs at {bad.size} of {g.size}, first {bad[:5]}: "
                                 f"got {g[bad[:5]]} want {w[bad[:5]]}")


def make(kind, n, sigma, rng):
    if kind == "uniform":
        return rng.integers(0, sigma, n).astype(np.uint8)
    if kind == "zipf":
        ranks = np.minimum(rng.zipf(1.3, n) - 1, sigma - 1)
        return rng.permutation(sigma)[ranks].astype(np.uint8)
    if kind == "sorted":
        return np.sort(rng.integers(0, sigma, n)).astype(np.uint8)
    if kind == "constant":
        return np.full(n, sigma - 1, dtype=np.uint8)
    if kind == "extremes":
        return np.where(rng.random(n) < 0.5, 0, sigma - 1).astype(np.uint8)
    if kind == "gaps":  # only even symbols: every odd leaf and many nodes empty
        return (2 * rng.integers(0, (sigma + 1) // 2, n)).astype(np.uint8)
    raise KeyError(kind)


SIZES = [1, 15, 16, 100, 4095, 16383, 16384, 16385, 3 * 16384 + 5, (1 << 20) + 7]
SIGMAS = [2, 3, 5, 64, 146, 255, 256]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("sigma", SIGMAS)
def test_uniform_sizes(wtmod, oracle_mod, n, sigma):
    S = make("uniform", n, sigma, np.random.default_rng(n * 7 + sigma))
    assert wtmod.histogram_path(n, sigma, 1) == wtmod.HIST_LEVELS
    t = wtmod.build(wtmod.to_device(S), sigma)
    torch.cuda.synchronize()
    assert t.status() == wtmod.WT_OK
    assert_same(t.to_numpy(), oracle_mod.build_all(S, sigma), f"uniform n={n} sigma={sigma}")


@pytest.mark.parametrize("kind", ["zipf", "sorted", "constant", "extremes", "gaps"])
@pytest.mark.parametrize("n,sigma", [(50_001, 256), (200_003, 146), (2_000_001, 256), (70_000, 2)])
def test_structured(wtmod, oracle_mod, kind, n, sigma):
    S = make(kind, n, sigma, np.random.default_rng(n + sigma))
    t = wtmod.build(wtmod.to_device(S), sigma)
    torch.cuda.synchronize()
    assert t.status() == wtmod.WT_OK
    assert_same(t.to_numpy(), oracle_mod.build_all(S, sigma), f"{kind} n={n} sigma={sigma}")


def test_text_like(wtmod, oracle_mod):
    S = inputs.text_like(3_000_017)
    say("[stats] text-like n=3000017")
    t = wtmod.build(wtmod.to_device(S), 256)
    torch.cuda.synchronize()
    assert t.status() == wtmod.WT_OK
    assert_same(t.to_numpy(), oracle_mod.build_all(S, 256), "text-like")


@pytest.mark.parametrize("sigma", [5, 146, 255])
def test_symbol_check(wtmod, sigma):
    n = 100_003
    for pos in (0, 54_321, n - 1):
        S = np.random.default_rng(pos).integers(0, sigma, n).astype(np.uint8)
        S[pos] = sigma
        t = wtmod.build(wtmod.to_device(S), sigma)
        torch.cuda.synchronize()
        assert t.status() == wtmod.WT_ERR_SYMBOL, (sigma, pos)
    S = np.full(n, sigma - 1, dtype=np.uint8)
    t = wtmod.build(wtmod.to_device(S), sigma)
    torch.cuda.synchronize()
    assert t.status() == wtmod.WT_OK


def test_rebuild_after_rejection(wtmod, oracle_mod):
    """The status word and every counter are rewritten by the next build
    into the same buffers."""
    n, sigma = 300_001, 100
    S = np.random.default_rng(9).integers(0, sigma, n).astype(np.uint8)
    bad = S.copy()
    bad[n // 2] = 200
    t = wtmod.WaveletTree.allocate(n, sigma, 1)
    t.build_from(wtmod.to_device(bad))
    torch.cuda.synchronize()
    assert t.status() == wtmod.WT_ERR_SYMBOL
    t.build_from(wtmod.to_device(S))
    torch.cuda.synchronize()
    assert t.status() == wtmod.WT_OK
    assert_same(t.to_numpy(), oracle_mod.build_all(S, sigma), "after a rejected build")


@pytest.mark.parametrize("n,sigma", [(16385, 2), (100_000, 3), (1_000_003, 256), (3 * 16384, 146)])
def test_without_directories(wtmod, oracle_mod, n, sigma):
    """No directories: the last level's bits come from level L-2's pass
    alone (no directory pass runs)."""
    S = make("zipf", n, sigma, np.random.default_rng(n))
    t = wtmod.build(wtmod.to_device(S), sigma, directories=False)
    torch.cuda.synchronize()
    assert t.status() == wtmod.WT_OK
    want = oracle_mod.build(S, sigma)
    got = t.to_numpy()
    for k in ("bits", "C"):
        assert np.array_equal(np.asarray(got[k], np.uint64).reshape(-1), np.asarray(want[k], np.uint64).reshape(-1)), k
