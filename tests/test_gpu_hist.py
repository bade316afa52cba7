"""GPU parity of the wide-alphabet histogram (sigma > 8192): the sliced LDS
path (2^16-symbol slices of packed 16-bit counters, one row of counts per
input chunk) and the LDS-hash path give C, and the whole tree, equal to the
oracle's.  The cases sit in the sliced regime: the sequence ping-pong of the
scratch (n times the level width) holds at least one row of sigma 32-bit
counts.  Integer work: tolerance zero."""
import sys

import numpy as np
import pytest

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
    yield wt
    wt.set_sliced_histogram(True)


def assert_same(got, want, ctx):
    for k in KEYS:
        g = np.asarray(got[k], dtype=np.uint64).reshape(-1)
        w = np.asarray(want[k], dtype=np.uint64).reshape(-1)
        assert g.shape == w.shape, (ctx, k, g.shape, w.shape)
        if not np.array_equal(g, w):
            bad = np.flatnonzero(g != w)
            raise AssertionError(f"{ctx}: {k} differs at {bad.size} of {g.size}, first {bad[:5]}: "
                                 f"got {g[bad[:5]]} want {w[bad[:5]]}")


def case_input(name):
    rng = np.random.default_rng(8142)
    if name == "u16_sigma8193_ragged":
        return rng.integers(0, 8193, 1_000_003).astype(np.uint16), 8193
    if name == "u16_heavy_symbol":
        # one symbol at 80%: its 16-bit LDS counter hands 2^15 on to the
        # global count several times in every chunk
        n = (1 << 20) + 5
        S = np.where(rng.random(n) < 0.8, 7, rng.integers(0, 40000, n)).astype(np.uint16)
        return S, 40000
    if name == "u16_sigma65536":
        return rng.integers(0, 1 << 16, 1 << 21).astype(np.uint16), 1 << 16
    if name == "u32_two_slices":
        # sigma = 2^16 + 1: the second slice holds one symbol, made heavy
        n = 5 << 20
        r = rng.random(n)
        S = rng.integers(0, (1 << 16) + 1, n).astype(np.uint32)
        S[r < 0.3] = 1 << 16
        S[(r >= 0.3) & (r < 0.35)] = (1 << 16) - 1
        return S, (1 << 16) + 1
    if name == "u32_17_slices":
        # 2^20 + 7 symbols: 17 slices, the last one 7 symbols wide; Zipf-like
        n = 3 << 20
        sigma = (1 << 20) + 7
        ranks = np.minimum(rng.zipf(1.3, n) - 1, sigma - 1)
        perm = rng.permutation(sigma)
        return perm[ranks].astype(np.uint32), sigma
    if name == "u32_sigma2p20":
        return rng.integers(0, 1 << 20, (1 << 21) + 3).astype(np.uint32), 1 << 20
    raise KeyError(name)


CASES = ["u16_sigma8193_ragged", "u16_heavy_symbol", "u16_sigma65536", "u32_two_slices", "u32_17_slices",
         "u32_sigma2p20"]


@pytest.mark.parametrize("case", CASES)
def test_wide_histogram_paths_match_oracle(wtmod, oracle_mod, case):
    S, sigma = case_input(case)
    say(f"[hist] {case}: n={S.size} sigma={sigma} {S.dtype}")
    want = oracle_mod.build_all(S, sigma)
    d = wtmod.to_device(S)
    outs = {}
    for sliced in (True, False):
        wtmod.set_sliced_histogram(sliced)
        t = wtmod.build(d, sigma)
        torch.cuda.synchronize()
        assert t.status() == wtmod.WT_OK, (case, sliced)
        outs[sliced] = t.to_numpy()
        assert_same(outs[sliced], want, f"{case} sliced={sliced}")
    wtmod.set_sliced_histogram(True)


@pytest.mark.parametrize("dtype,sigma,n", [(np.uint16, 40000, 1 << 20), (np.uint32, (1 << 20) + 7, 3 << 20)])
def test_wide_histogram_rejects_symbol(wtmod, dtype, sigma, n):
    """A symbol >= sigma is reported by both paths (wherever it sits: the
    first position, the last of a ragged input)."""
    rng = np.random.default_rng(5)
    for pos in (0, n - 1):
        S = rng.integers(0, sigma, n).astype(dtype)
        S[pos] = sigma
        for sliced in (True, False):
            wtmod.set_sliced_histogram(sliced)
            t = wtmod.build(wtmod.to_device(S), sigma)
            torch.cuda.synchronize()
            assert t.status() == wtmod.WT_ERR_SYMBOL, (dtype, sigma, pos, sliced)
    wtmod.set_sliced_histogram(True)
