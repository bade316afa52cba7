"""GPU parity of the 4-ary wavelet tree (wt_build_multiary, byte symbols)
against the oracle's multiary tree, bit for bit: the 2-bit entries of every
level, C and the digit directories; queries against naive counting over S.
Integer work: tolerance zero."""
import sys

import numpy as np
import pytest

from paper_1407_8142_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIZES = [0, 1, 2, 31, 32, 33, 511, 512, 513, 4095, 4096, 4097, 16383, 16384, 16385, 69635, 200001]
KEYS = ("digits", "C", "rank4", "sel4", "counts4")


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


def assert_same(got, want, ctx):
    for k in KEYS:
        g = np.asarray(got[k], dtype=np.uint64).reshape(-1)
        w = np.asarray(want[k], dtype=np.uint64).reshape(-1)
        assert g.shape == w.shape, (ctx, k, g.shape, w.shape)
        if not np.array_equal(g, w):
            bad = np.flatnonzero(g != w)
            raise AssertionError(f"{ctx}: {k} differs at {bad.size} of {g.size}, first {bad[:5]}: "
                                 f"got {g[bad[:5]]} want {w[bad[:5]]}")


def check(wt, oracle_mod, S, sigma, ctx):
    want = oracle_mod.build_multiary_all(S, sigma)
    t = wt.build_multiary(wt.to_device(S), sigma)
    torch.cuda.synchronize()
    assert t.status() == wt.WT_OK, ctx
    assert_same(t.to_numpy(), want, ctx)
    return t


@pytest.mark.parametrize("sigma", [1, 2, 3, 4, 5, 8, 16, 100, 146, 255, 256])
def test_multiary_sizes(wtmod, oracle_mod, sigma):
    rng = np.random.default_rng(700 + sigma)
    for n in SIZES:
        say(f"[multiary] n={n} sigma={sigma}")
        check(wtmod, oracle_mod, rng.integers(0, sigma, n).astype(np.uint8), sigma, f"n={n} sigma={sigma}")


@pytest.mark.parametrize("case", ["sorted", "reverse", "constant", "runs", "geometric", "two_far", "text"])
def test_multiary_inputs(wtmod, oracle_mod, case):
    rng = np.random.default_rng(71)
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
        S, sigma = np.minimum(rng.geometric(0.03, n) - 1, 255).astype(np.uint8), 256
    elif case == "two_far":
        S, sigma = np.where(rng.random(n) < 0.5, 0, 255).astype(np.uint8), 256
    else:
        S, sigma = inputs.text_like(1 << 22), 256
    say(f"[multiary] {case}: n={S.size} sigma={sigma}")
    check(wtmod, oracle_mod, S, sigma, case)


def _naive_rank(S, c, i):
    return int(np.count_nonzero(S[: min(i, S.size)] == c))


def _naive_select(S, c, k):
    if k <= 0:
        return -1
    pos = np.flatnonzero(S == c)
    return int(pos[k - 1]) if k <= pos.size else -1


@pytest.mark.parametrize("n,sigma", [(9, 5), (10, 16), (70001, 256), (50000, 3), (30000, 7), (1000, 1)])
def test_multiary_queries(wtmod, oracle_mod, n, sigma):
    rng = np.random.default_rng(n + sigma)
    S = rng.integers(0, sigma, n).astype(np.uint8)
    t = check(wtmod, oracle_mod, S, sigma, f"queries n={n} sigma={sigma}")
    dev = torch.device("cuda")
    if n <= 16:
        qi = np.arange(n + 2)
        cs = np.repeat(np.arange(sigma + 1), n + 2)
        js = np.tile(np.arange(n + 2), sigma + 1)
    else:
        qi = rng.integers(0, n + 3, 4000)
        cs = np.where(rng.random(4000) < 0.8, S[rng.integers(0, n, 4000)], rng.integers(0, sigma + 2, 4000))
        js = rng.integers(0, n + 3, 4000)
    acc = t.access(torch.from_numpy(qi).to(dev)).cpu().numpy().view(np.uint32)
    S64 = S.astype(np.int64)
    want = np.where(qi < n, S64[np.minimum(qi, n - 1)] if n else 0, 0xFFFFFFFF).astype(np.uint32)
    assert np.array_equal(acc, want)
    rk = t.rank_query(torch.from_numpy(cs.astype(np.int32)).to(dev), torch.from_numpy(js).to(dev)).cpu().numpy()
    assert all(int(rk[q]) == (_naive_rank(S, int(cs[q]), int(js[q])) if cs[q] < sigma else 0)
               for q in range(cs.size))
    ks = js % (n // max(sigma, 1) + 3) if n > 16 else js
    sl = t.select_query(torch.from_numpy(cs.astype(np.int32)).to(dev), torch.from_numpy(ks).to(dev)).cpu().numpy()
    assert all(int(sl[q]) == (_naive_select(S, int(cs[q]), int(ks[q])) if cs[q] < sigma else -1)
               for q in range(cs.size))


def test_multiary_rejects(wtmod):
    S = np.random.default_rng(73).integers(0, 100, 50000).astype(np.uint8)
    S[777] = 100
    t = wtmod.build_multiary(wtmod.to_device(S), 100)
    torch.cuda.synchronize()
    assert t.status() == wtmod.WT_ERR_SYMBOL
