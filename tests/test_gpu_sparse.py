"""GPU parity of builds whose node tables cover only the nonempty nodes
(32-bit alphabets much larger than the sequence, and sigma up to 2^32, L up
to 32): every output buffer (bits, C, rank, sel1, sel0, sel_counts) equals
the oracle's, bit for bit (integer work: tolerance zero); the wavelet matrix
of such an alphabet too; queries on the tree against naive counting over S;
a rejected symbol; n = 0.  C is dense (sigma + 1 entries, 16 or 32 GiB at
the largest alphabets) and compared in slices."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("bits", "rank", "sel1", "sel0", "sel_counts")


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


def same_C(C_dev, C_want, ctx):
    step = 1 << 28
    for a in range(0, C_want.size, step):
        g = C_dev[a:a + step].cpu().numpy().view(np.uint64)
        w = C_want[a:a + step]
        if not np.array_equal(g, w):
            bad = np.flatnonzero(g != w)
            raise AssertionError(f"{ctx}: C differs at {bad.size} entries from {a + bad[0]}")


def same(t, want, ctx):
    same_C(t.C, want["C"], ctx)
    got = {k: getattr(t, k).cpu().numpy().view(np.uint64) for k in KEYS}
    for k in KEYS:
        g = got[k].reshape(-1)
        w = np.asarray(want[k], dtype=np.uint64).reshape(-1)
        assert g.shape == w.shape, (ctx, k)
        bad = np.flatnonzero(g != w)
        assert bad.size == 0, f"{ctx}: {k} differs at {bad.size} of {g.size}, first {bad[:5]}"


def build_check(wt, oracle_mod, S, sigma, ctx):
    lay = wt.plan(S.size, sigma, 4)
    say(f"[sparse] {ctx}: n={S.size} sigma={sigma} L={lay.L} scratch={lay.scratch_bytes >> 20} MiB")
    t = wt.build(wt.to_device(S), sigma)
    torch.cuda.synchronize()
    assert t.status() == wt.WT_OK
    say(f"[sparse] {ctx}: oracle")
    want = oracle_mod.build_all(S, sigma)
    same(t, want, ctx)
    say(f"[sparse] {ctx}: equal")
    return t


def test_small_n_wide_alphabet(wtmod, oracle_mod):
    rng = np.random.default_rng(12)
    S = rng.integers(0, 1 << 20, 1 << 12).astype(np.uint32)
    build_check(wtmod, oracle_mod, S, 1 << 20, "sigma=2^20 n=2^12")


@pytest.mark.parametrize("n,sigma,kind", [
    ((1 << 20) + 5, 1 << 24, "uniform"),        # tiles span thousands of nodes at deep levels
    ((1 << 21) + 3, 1 << 28, "zipf"),
    (300_001, (1 << 25) + 1, "clustered"),      # many empty subtrees, one symbol past the last power of two
])
def test_sparse_shapes(wtmod, oracle_mod, n, sigma, kind):
    rng = np.random.default_rng(n ^ sigma)
    if kind == "uniform":
        S = rng.integers(0, sigma, n, dtype=np.uint64).astype(np.uint32)
    elif kind == "zipf":
        ranks = np.minimum(rng.zipf(1.2, n) - 1, (1 << 20) - 1)
        ids = rng.integers(0, sigma, 1 << 20, dtype=np.uint64)
        S = ids[ranks].astype(np.uint32)
    else:
        S = (rng.integers(0, 64, n) * 524_288 + rng.integers(0, 3, n)).astype(np.uint32)
        S[::1000] = sigma - 1
    build_check(wtmod, oracle_mod, S, sigma, f"{kind} n={n} sigma={sigma}")


def queries(wt, t, S, rng):
    n = S.size
    i = rng.integers(0, n, 2000)
    acc = t.access(torch.from_numpy(i).cuda()).cpu().numpy().view(np.uint32)
    assert np.array_equal(acc, S[i])
    cs = np.concatenate([S[rng.integers(0, n, 20)], [0, (1 << 32) - 1]]).astype(np.uint64)
    for c in cs:
        pos = np.flatnonzero(S == c)
        ii = np.array([0, n // 3, n], dtype=np.int64)
        r = t.rank_query(torch.tensor([int(c) - (1 << 32) if c >= (1 << 31) else int(c)] * 3, dtype=torch.int64).cuda(),
                         torch.from_numpy(ii).cuda()).cpu().numpy()
        assert list(r) == [int(np.count_nonzero(pos < x)) for x in ii], c
        if pos.size:
            k = np.array([1, pos.size], dtype=np.int64)
            sel = t.select_query(torch.tensor([int(c) - (1 << 32) if c >= (1 << 31) else int(c)] * 2,
                                              dtype=torch.int64).cuda(), torch.from_numpy(k).cuda()).cpu().numpy()
            assert list(sel) == [int(pos[0]), int(pos[-1])], c


def test_sigma_2p31_plus_1(wtmod, oracle_mod):
    rng = np.random.default_rng(31)
    n, sigma = 100_003, (1 << 31) + 1
    S = rng.integers(0, sigma, n, dtype=np.uint64).astype(np.uint32)
    S[5] = sigma - 1
    t = build_check(wtmod, oracle_mod, S, sigma, "sigma=2^31+1")
    queries(wtmod, t, S, rng)
    del t
    torch.cuda.empty_cache()


def test_sigma_2p32(wtmod, oracle_mod):
    rng = np.random.default_rng(32)
    n, sigma = 65_537, 1 << 32
    S = rng.integers(0, sigma, n, dtype=np.uint64).astype(np.uint32)
    S[:3] = [(1 << 32) - 1, 0, (1 << 31)]
    S[-1] = (1 << 32) - 1
    t = build_check(wtmod, oracle_mod, S, sigma, "sigma=2^32")
    queries(wtmod, t, S, rng)
    del t
    torch.cuda.empty_cache()


def test_matrix_wide_alphabet(wtmod, oracle_mod):
    rng = np.random.default_rng(7)
    n, sigma = 70_001, (1 << 26) + 3
    S = rng.integers(0, sigma, n, dtype=np.uint64).astype(np.uint32)
    m = wtmod.build_matrix(wtmod.to_device(S), sigma)
    torch.cuda.synchronize()
    assert m.status() == wtmod.WT_OK
    want = oracle_mod.build_matrix_all(S, sigma)
    t = m.tree
    for k in ("bits", "rank", "sel1", "sel0", "sel_counts"):
        g = getattr(t, k).cpu().numpy().view(np.uint64).reshape(-1)
        w = np.asarray(want[k], dtype=np.uint64).reshape(-1)
        assert np.array_equal(g, w), k
    assert np.array_equal(m.zeros.cpu().numpy().view(np.uint64)[:t.L], np.asarray(want["zeros"], dtype=np.uint64))


def test_rejected_symbol_and_empty(wtmod):
    n, sigma = 50_000, (1 << 31) + 1
    S = np.random.default_rng(1).integers(0, 1 << 30, n).astype(np.uint32)
    S[n // 2] = (1 << 31) + 1
    t = wtmod.build(wtmod.to_device(S), sigma)
    torch.cuda.synchronize()
    assert t.status() == wtmod.WT_ERR_SYMBOL
    del t
    torch.cuda.empty_cache()
    e = wtmod.build(torch.empty(0, dtype=torch.int32, device="cuda"), (1 << 25) + 1)
    torch.cuda.synchronize()
    assert e.status() == wtmod.WT_OK
    assert int(e.C.abs().sum().item()) == 0
    assert e.sel_counts.abs().sum().item() == 0
