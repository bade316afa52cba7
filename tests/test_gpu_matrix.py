"""GPU parity of the wavelet matrix (wt_build_matrix and the matrix queries)
against the oracle's matrix, bit for bit: level bitmaps, per-level zero
counts, C and the directories; queries against naive counting over S.
Integer work: tolerance zero."""
import sys

import numpy as np
import pytest

from paper_1407_8142_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIZES = [0, 1, 2, 63, 64, 65, 511, 512, 513, 4095, 4096, 4097, 16383, 16384, 16385, 69635]


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


def assert_same(got, want, ctx, keys=("bits", "zeros", "rank", "sel1", "sel0", "sel_counts")):
    for k in keys:
        g = np.asarray(got[k], dtype=np.uint64).reshape(-1)
        w = np.asarray(want[k], dtype=np.uint64).reshape(-1)
        assert g.shape == w.shape, (ctx, k, g.shape, w.shape)
        if not np.array_equal(g, w):
            bad = np.flatnonzero(g != w)
            raise AssertionError(f"{ctx}: {k} differs at {bad.size} of {g.size}, first {bad[:5]}: "
                                 f"got {g[bad[:5]]} want {w[bad[:5]]}")


def check(wt, oracle_mod, S, sigma, ctx):
    want = oracle_mod.build_matrix_all(S, sigma)
    m = wt.build_matrix(wt.to_device(S), sigma)
    torch.cuda.synchronize()
    assert m.status() == wt.WT_OK, ctx
    got = m.to_numpy()
    assert_same(got, want, ctx)
    assert np.array_equal(got["C"], oracle_mod.build(S, sigma)["C"]), ctx
    return m


@pytest.mark.parametrize("sigma", [1, 2, 3, 5, 146, 256])
def test_matrix_u8_sizes(wtmod, oracle_mod, sigma):
    rng = np.random.default_rng(500 + sigma)
    for n in SIZES:
        say(f"[matrix] n={n} sigma={sigma}")
        check(wtmod, oracle_mod, rng.integers(0, sigma, n).astype(np.uint8), sigma, f"n={n} sigma={sigma}")


@pytest.mark.parametrize("case", ["u16_small", "u16_full", "u32_wide", "u32_narrow", "sorted", "constant",
                                  "two_runs", "text"])
def test_matrix_inputs(wtmod, oracle_mod, case):
    rng = np.random.default_rng(91)
    if case == "u16_small":
        S, sigma = rng.integers(0, 300, 50001).astype(np.uint16), 300
    elif case == "u16_full":
        S, sigma = rng.integers(0, 1 << 16, 120000).astype(np.uint16), 1 << 16
    elif case == "u32_wide":
        S, sigma = rng.integers(0, (1 << 20) + 7, 90001).astype(np.uint32), (1 << 20) + 7
    elif case == "u32_narrow":
        S, sigma = rng.integers(0, 60, 77777).astype(np.uint32), 60
    elif case == "sorted":
        S, sigma = np.sort(rng.integers(0, 256, 100000)).astype(np.uint8), 256
    elif case == "constant":
        S, sigma = np.full(40000, 77, np.uint8), 128
    elif case == "two_runs":
        S, sigma = np.concatenate([np.full(30000, 200, np.uint8), np.full(30001, 3, np.uint8)]), 256
    else:
        S, sigma = inputs.text_like(1 << 22), 256
    say(f"[matrix] {case}: n={S.size} sigma={sigma}")
    check(wtmod, oracle_mod, S, sigma, case)


def _naive_rank(S, c, i):
    return int(np.count_nonzero(S[: min(i, S.size)] == c))


def _naive_select(S, c, k):
    if k <= 0:
        return -1
    pos = np.flatnonzero(S == c)
    return int(pos[k - 1]) if k <= pos.size else -1


@pytest.mark.parametrize("n,sigma,dtype", [(9, 5, np.uint8), (70001, 256, np.uint8), (50000, 3, np.uint8),
                                           (40000, 1 << 16, np.uint16), (30000, (1 << 20) + 3, np.uint32),
                                           (1000, 1, np.uint8)])
def test_matrix_queries(wtmod, oracle_mod, n, sigma, dtype):
    rng = np.random.default_rng(n + sigma)
    S = rng.integers(0, sigma, n).astype(dtype)
    m = check(wtmod, oracle_mod, S, sigma, f"queries n={n} sigma={sigma}")
    dev = torch.device("cuda")
    if n <= 16:
        qi = np.arange(n + 2)
        cs = np.repeat(np.arange(sigma + 1), n + 2)
        js = np.tile(np.arange(n + 2), sigma + 1)
    else:
        qi = rng.integers(0, n + 3, 4000)
        cs = np.where(rng.random(4000) < 0.8, S[rng.integers(0, n, 4000)], rng.integers(0, sigma + 2, 4000))
        js = rng.integers(0, n + 3, 4000)
    acc = m.access(torch.from_numpy(qi).to(dev)).cpu().numpy().view(np.uint32)
    S64 = S.astype(np.int64)
    want = np.where(qi < n, S64[np.minimum(qi, n - 1)] if n else 0, 0xFFFFFFFF).astype(np.uint32)
    assert np.array_equal(acc, want)
    rk = m.rank_query(torch.from_numpy(cs.astype(np.int32)).to(dev), torch.from_numpy(js).to(dev)).cpu().numpy()
    assert all(int(rk[q]) == _naive_rank(S, int(cs[q]), int(js[q])) for q in range(cs.size))
    ks = js % (n // max(sigma, 1) + 3) if n > 16 else js
    sl = m.select_query(torch.from_numpy(cs.astype(np.int32)).to(dev), torch.from_numpy(ks).to(dev)).cpu().numpy()
    assert all(int(sl[q]) == (_naive_select(S, int(cs[q]), int(ks[q])) if cs[q] < sigma else -1)
               for q in range(cs.size))


def test_matrix_rejects_symbol(wtmod):
    S = np.random.default_rng(93).integers(0, 100, 50000).astype(np.uint8)
    S[12345] = 100
    m = wtmod.build_matrix(wtmod.to_device(S), 100)
    torch.cuda.synchronize()
    assert m.status() == wtmod.WT_ERR_SYMBOL
