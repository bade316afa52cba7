"""GPU parity of the two-levels-per-pass build for byte alphabets (switched
on here; one level per pass is the default): with the fused tail levels
switched off every byte input of n >= 1 and L >= 2 runs through the pair
passes (levels l and l+1 from one read of S_l), and every output buffer must
equal the oracle's, as it must with one level per pass.
Integer work: tolerance zero."""
import sys

import numpy as np
import pytest

from paper_1407_8142_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("bits", "C", "rank", "sel1", "sel0", "sel_counts")
SIZES = [1, 2, 63, 64, 65, 511, 512, 513, 4095, 4096, 4097, 16383, 16384, 16385, 40000, 69635, 200001]


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
    prev = wt.set_level_pairs(False)
    yield wt
    wt.set_fused_levels(True)
    wt.set_level_pairs(prev)


def assert_same(got, want, ctx, keys=KEYS):
    for k in keys:
        g = np.asarray(got[k], dtype=np.uint64).reshape(-1)
        w = np.asarray(want[k], dtype=np.uint64).reshape(-1)
        assert g.shape == w.shape, (ctx, k, g.shape, w.shape)
        if not np.array_equal(g, w):
            bad = np.flatnonzero(g != w)
            raise AssertionError(f"{ctx}: {k} differs at {bad.size} of {g.size}, first {bad[:5]}: "
                                 f"got {g[bad[:5]]} want {w[bad[:5]]}")


def build_both(wt, oracle_mod, S, sigma, ctx, directories=True):
    want = oracle_mod.build_all(S, sigma)
    d = wt.to_device(S)
    for pairs in (True, False):
        wt.set_level_pairs(pairs)
        t = wt.build(d, sigma, directories=directories)
        torch.cuda.synchronize()
        assert t.status() == wt.WT_OK, (ctx, pairs)
        keys = KEYS if directories else ("bits", "C")
        assert_same(t.to_numpy(), want, f"{ctx} pairs={pairs}", keys)
    wt.set_level_pairs(False)


@pytest.mark.parametrize("sigma", [2, 3, 4, 5, 16, 146, 255, 256])
def test_pairs_size_sweep(wtmod, oracle_mod, sigma):
    rng = np.random.default_rng(1000 + sigma)
    for n in SIZES:
        S = rng.integers(0, sigma, n).astype(np.uint8)
        say(f"[pairs] n={n} sigma={sigma}")
        build_both(wtmod, oracle_mod, S, sigma, f"n={n} sigma={sigma}")


@pytest.mark.parametrize("case", ["sorted", "reverse", "constant", "runs", "geometric", "two_symbols_far",
                                  "alternating", "text"])
def test_pairs_structured(wtmod, oracle_mod, case):
    rng = np.random.default_rng(77)
    n = 150001
    if case == "sorted":
        S, sigma = np.sort(rng.integers(0, 256, n)).astype(np.uint8), 256
    elif case == "reverse":
        S, sigma = np.sort(rng.integers(0, 200, n))[::-1].astype(np.uint8).copy(), 200
    elif case == "constant":
        S, sigma = np.full(n, 99, np.uint8), 128
    elif case == "runs":
        S = np.repeat(rng.integers(0, 256, 9000), rng.integers(1, 40, 9000)).astype(np.uint8)
        sigma = 256
    elif case == "geometric":
        # node sizes of every magnitude, many tiny nodes in one tile
        S, sigma = np.minimum(rng.geometric(0.03, n) - 1, 255).astype(np.uint8), 256
    elif case == "two_symbols_far":
        S, sigma = np.where(rng.random(n) < 0.5, 0, 255).astype(np.uint8), 256
    elif case == "alternating":
        S, sigma = (np.arange(n) % 2 * 170 + 3).astype(np.uint8), 256
    else:
        S, sigma = inputs.text_like(1 << 21), 256
    say(f"[pairs] {case}: n={S.size} sigma={sigma}")
    build_both(wtmod, oracle_mod, S, sigma, case)


def test_pairs_without_directories(wtmod, oracle_mod):
    rng = np.random.default_rng(5)
    for n, sigma in [(70001, 256), (33333, 7), (16385, 4)]:
        S = rng.integers(0, sigma, n).astype(np.uint8)
        build_both(wtmod, oracle_mod, S, sigma, f"no dirs n={n} sigma={sigma}", directories=False)


def test_pairs_reject_symbol(wtmod):
    S = np.random.default_rng(6).integers(0, 100, 50000).astype(np.uint8)
    S[40000] = 100
    wtmod.set_level_pairs(True)
    try:
        t = wtmod.build(wtmod.to_device(S), 100)
        torch.cuda.synchronize()
        assert t.status() == wtmod.WT_ERR_SYMBOL
    finally:
        wtmod.set_level_pairs(False)
