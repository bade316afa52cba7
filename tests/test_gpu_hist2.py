"""Two-phase histogram of wide alphabets (trees of more than 16 levels over
32-bit symbols, n >= 2^20): counts of the top L-16 bits before level 0, the
low 16 bits per segment of S_{L-16} after level L-17.  Every output equals
the oracle's (integer work, tolerance zero) and the hashing path's, also
where segments are empty, where a block's share spans several segments,
and where a 16-bit LDS counter overflows many times."""
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
    return wt


def build_np(wt, S, sigma):
    t = wt.build(wt.to_device(S), sigma)
    torch.cuda.synchronize()
    assert t.status() == wt.WT_OK
    return t.to_numpy()


def build_hashing(wt, S, sigma):
    wt.set_sliced_histogram(False)
    try:
        return build_np(wt, S, sigma)
    finally:
        wt.set_sliced_histogram(True)


def same(got, want, ctx):
    for k in KEYS:
        g = np.asarray(got[k], dtype=np.uint64).reshape(-1)
        w = np.asarray(want[k], dtype=np.uint64).reshape(-1)
        assert g.shape == w.shape and np.array_equal(g, w), (ctx, k, np.flatnonzero(g != w)[:5])


def zipf_ids(rng, n, sigma, s=1.0):
    ranks = np.minimum(rng.zipf(1.0 + s, n) - 1, sigma - 1).astype(np.int64)
    perm = rng.permutation(sigma)
    return perm[ranks].astype(np.uint32)


CASES = [
    ("uniform sigma=2^20, ragged n", (1 << 20) + 4099, 1 << 20, "uniform"),
    ("Zipf sigma=2^20+3 (21 levels, 32 groups, most empty)", 1 << 21, (1 << 20) + 3, "zipf"),
    ("half uniform, half Zipf sigma=2^17 (one coarse bit)", 3 * (1 << 20) + 5, 1 << 17, "mix"),
    ("one group holds everything (sigma=2^20)", (1 << 20) + 77, 1 << 20, "onegroup"),
]


def make(kind, n, sigma, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.integers(0, sigma, n).astype(np.uint32)
    if kind == "zipf":
        return zipf_ids(rng, n, sigma)
    if kind == "mix":
        S = np.concatenate([rng.integers(0, sigma, n // 2).astype(np.uint32), zipf_ids(rng, n - n // 2, sigma)])
        return S
    base = 5 << 16
    return (base + rng.integers(0, 100, n)).astype(np.uint32)


@pytest.mark.parametrize("ctx,n,sigma,kind", CASES, ids=[c[3] for c in CASES])
def test_two_phase_equals_oracle(wtmod, oracle_mod, ctx, n, sigma, kind):
    say(f"[hist2] {ctx}: n={n} sigma={sigma}")
    S = make(kind, n, sigma, n ^ sigma)
    got = build_np(wtmod, S, sigma)
    assert np.array_equal(np.asarray(got["C"], dtype=np.uint64),
                          np.concatenate([[0], np.cumsum(np.bincount(S, minlength=sigma))]).astype(np.uint64))
    same(got, oracle_mod.build_all(S, sigma), ctx)


def test_two_phase_counter_overflow(wtmod):
    # 2^24 symbols, 70% one symbol: each block's share holds ~45000 copies,
    # so its 16-bit LDS counter hands 2^15 to the overflow counts.
    n, sigma = 1 << 24, 1 << 20
    say(f"[hist2] overflow: n={n} sigma={sigma}")
    rng = np.random.default_rng(24)
    S = rng.integers(0, sigma, n).astype(np.uint32)
    S[rng.random(n) < 0.7] = 777777
    got = build_np(wtmod, S, sigma)
    assert np.array_equal(np.asarray(got["C"], dtype=np.uint64),
                          np.concatenate([[0], np.cumsum(np.bincount(S, minlength=sigma))]).astype(np.uint64))
    same(got, build_hashing(wtmod, S, sigma), "overflow")


def test_two_phase_rejects_bad_symbol(wtmod):
    n, sigma = (1 << 20) + 9, (1 << 18) + 1
    say(f"[hist2] bad symbol: n={n} sigma={sigma}")
    rng = np.random.default_rng(7)
    S = rng.integers(0, sigma, n).astype(np.uint32)
    S[12345] = sigma + 5
    t = wtmod.build(wtmod.to_device(S), sigma)
    torch.cuda.synchronize()
    assert t.status() != wtmod.WT_OK
