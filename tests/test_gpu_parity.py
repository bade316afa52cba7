"""GPU parity: every output buffer of wt_build (bits, C, rank, sel1, sel0,
sel_counts) equals the oracle's, bit for bit; queries equal naive counting.
Integer work throughout, so the tolerance is zero."""
import sys

import numpy as np
import pytest

import pins
from paper_1407_8142_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def gpu_build(wt, S, sigma, directories=True):
    d = wt.to_device(S)
    t = wt.build(d, sigma, directories=directories)
    torch.cuda.synchronize()
    assert t.status() == wt.WT_OK
    return t


def assert_same(got: dict, want: dict, keys=("bits", "C", "rank", "sel1", "sel0", "sel_counts"), ctx=""):
    for k in keys:
        g = np.asarray(got[k], dtype=np.uint64).reshape(-1)
        w = np.asarray(want[k], dtype=np.uint64).reshape(-1)
        assert g.shape == w.shape, (ctx, k, g.shape, w.shape)
        if not np.array_equal(g, w):
            bad = np.flatnonzero(g != w)
            raise AssertionError(f"{ctx}: {k} differs at {bad.size} of {g.size} entries, first {bad[:5]}: "
                                 f"got {g[bad[:5]]} want {w[bad[:5]]}")


def check_against_oracle(wt, oracle_mod, S, sigma, ctx):
    say(f"[parity] {ctx}: n={S.size} sigma={sigma} dtype={S.dtype}")
    t = gpu_build(wt, S, sigma)
    want = oracle_mod.build_all(S, sigma)
    assert_same(t.to_numpy(), want, ctx=ctx)
    return t, want


EDGE_N = [0, 1, 2, 63, 64, 65, 511, 512, 513, 4095, 4096, 4097, 8191, 8192, 12305, 65536 + 4096 + 3]


@pytest.mark.parametrize("n", EDGE_N)
@pytest.mark.parametrize("sigma", [1, 2, 3, 5, 146, 256])
def test_edge_sizes_u8(wtmod, oracle_mod, n, sigma):
    rng = np.random.default_rng(n * 1000 + sigma)
    S = rng.integers(0, sigma, n).astype(np.uint8)
    check_against_oracle(wtmod, oracle_mod, S, sigma, f"u8 n={n} sigma={sigma}")


@pytest.mark.parametrize("n", [1, 64, 4097, 50000])
@pytest.mark.parametrize("sigma,dtype", [(257, np.uint16), (1 << 16, np.uint16), (1000, np.uint32),
                                         ((1 << 16) + 1, np.uint32), (1 << 20, np.uint32), (3, np.uint32),
                                         (200, np.uint16)])
def test_edge_sizes_wide(wtmod, oracle_mod, n, sigma, dtype):
    rng = np.random.default_rng(n + sigma)
    S = rng.integers(0, sigma, n).astype(dtype)
    check_against_oracle(wtmod, oracle_mod, S, sigma, f"{np.dtype(dtype).name} n={n} sigma={sigma}")


@pytest.mark.parametrize("kind", ["all_equal_zero", "only_last", "sorted", "reverse_sorted", "sigma_gt_n",
                                  "alternating", "two_runs"])
def test_structured_inputs(wtmod, oracle_mod, kind):
    n, sigma = 20000, 256
    rng = np.random.default_rng(7)
    if kind == "all_equal_zero":
        S = np.zeros(n, np.uint8)
    elif kind == "only_last":
        S = np.full(n, sigma - 1, np.uint8)
    elif kind == "sorted":
        S = np.sort(rng.integers(0, sigma, n)).astype(np.uint8)
    elif kind == "reverse_sorted":
        S = np.sort(rng.integers(0, sigma, n))[::-1].astype(np.uint8).copy()
    elif kind == "sigma_gt_n":
        sigma = 1 << 16
        S = rng.integers(0, sigma, 3000).astype(np.uint16)
    elif kind == "alternating":
        S = (np.arange(n) % 2 * 255).astype(np.uint8)
    else:
        S = np.concatenate([np.full(4096 * 3 + 17, 3), np.full(n - 4096 * 3 - 17, 200)]).astype(np.uint8)
    check_against_oracle(wtmod, oracle_mod, S, sigma, kind)


def test_node_boundaries_on_word_block_tile_edges(wtmod, oracle_mod):
    # Node sizes chosen so level-1 and deeper boundaries land exactly on 64, 512 and 4096.
    parts = [(0, 64), (1, 448), (2, 3584), (3, 4096), (5, 1), (6, 63), (7, 4095), (9, 512)]
    S = np.concatenate([np.full(c, s) for s, c in parts]).astype(np.uint8)
    S = np.random.default_rng(3).permutation(S)
    check_against_oracle(wtmod, oracle_mod, np.sort(S).astype(np.uint8), 16, "aligned-sorted")
    check_against_oracle(wtmod, oracle_mod, S, 16, "aligned-shuffled")


def test_workload_uniform_full(wtmod, oracle_mod):
    S, sigma = inputs.workload("uniform256")
    check_against_oracle(wtmod, oracle_mod, S, sigma, "uniform n=2^20")


@pytest.mark.parametrize("cfg,n", [("text256", 1 << 22), ("alpha16", 1 << 21), ("alpha20", 1 << 21)])
def test_workloads_scaled(wtmod, oracle_mod, cfg, n):
    S, sigma = inputs.workload(cfg, n)
    check_against_oracle(wtmod, oracle_mod, S, sigma, f"{cfg} n={n}")


@pytest.mark.parametrize("n,sigma,dtype", [((4096 * 4096) + 4099, (1 << 17) + 3, np.uint32),
                                           ((4096 * 8192) + 12289, (1 << 16), np.uint16)])
def test_tile_prefixes_over_several_blocks(wtmod, oracle_mod, n, sigma, dtype):
    """Levels of more than 4096 tiles take their tile prefixes from the
    multi-block pass (a decoupled look-back between its blocks): 32-bit
    levels of 4096 symbols per tile and 16-bit levels of 8192, a ragged last
    tile and a ragged last block, against the oracle."""
    rng = np.random.default_rng(n)
    S = rng.integers(0, sigma, n).astype(dtype)
    check_against_oracle(wtmod, oracle_mod, S, sigma, f"multi-block tile prefixes n={n} sigma={sigma}")


def test_standalone_rank_select_matches(wtmod, oracle_mod):
    for n, sigma in [(0, 8), (1, 2), (4097, 5), (300001, 256), (70000, 1 << 20)]:
        rng = np.random.default_rng(n)
        S = rng.integers(0, sigma, n).astype(inputs.dtype_for_sigma(sigma))
        t = gpu_build(wtmod, S, sigma, directories=False)
        d = wtmod.build_rank_select(t.bits, n, t.L)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy().view(np.uint64) for k, v in d.items() if not k.startswith("_")}
        want = oracle_mod.rank_select(oracle_mod.build(S, sigma)["bits"], n, t.L)
        assert_same(got, want, keys=("rank", "sel1", "sel0", "sel_counts"), ctx=f"standalone n={n}")


def test_deterministic_rebuild(wtmod):
    S, sigma = inputs.workload("text256", 1 << 21)
    a = gpu_build(wtmod, S, sigma).to_numpy()
    b = gpu_build(wtmod, S, sigma).to_numpy()
    assert_same(a, b, ctx="rebuild")


def test_symbol_out_of_range_reported(wtmod):
    S = np.zeros(10000, np.uint8)
    S[7777] = 200
    d = wtmod.to_device(S)
    t = wtmod.build(d, 150)
    torch.cuda.synchronize()
    assert t.status() == wtmod.WT_ERR_SYMBOL
    # the same scratch is clean again after a valid build
    t.build_from(wtmod.to_device(np.zeros(10000, np.uint8)))
    assert t.status() == wtmod.WT_OK


def _queries_check(wt, t, S, sigma, rng, m=4000):
    n = S.size
    dev = "cuda"
    i = rng.integers(0, n + 3, m)
    got = t.access(torch.from_numpy(i).to(dev)).cpu().numpy().view(np.uint32)
    want = np.where(i < n, S[np.minimum(i, max(n - 1, 0))].astype(np.uint64) if n else 0, 0xFFFFFFFF)
    assert np.array_equal(got.astype(np.uint64), want.astype(np.uint64))
    c = np.where(rng.random(m) < 0.8, S[rng.integers(0, max(n, 1), m)] if n else 0,
                 rng.integers(0, sigma + 5, m)).astype(np.int64)
    ii = rng.integers(0, n + 2, m)
    got = t.rank_query(torch.from_numpy(c.astype(np.int32)).to(dev), torch.from_numpy(ii).to(dev)).cpu().numpy()
    # naive counting: per symbol, sorted positions
    order = np.argsort(S, kind="stable")
    starts = np.searchsorted(S[order], np.arange(sigma + 6))
    for q in range(m):
        cc, iq = int(c[q]), int(ii[q])
        pos = order[starts[cc]:starts[cc + 1]] if cc < sigma else np.zeros(0, np.int64)
        assert got[q] == np.searchsorted(pos, min(iq, n)), (q, cc, iq)
    k = rng.integers(0, 40, m)
    got = t.select_query(torch.from_numpy(c.astype(np.int32)).to(dev), torch.from_numpy(k).to(dev)).cpu().numpy()
    for q in range(m):
        cc, kq = int(c[q]), int(k[q])
        pos = order[starts[cc]:starts[cc + 1]] if cc < sigma else np.zeros(0, np.int64)
        want = int(pos[kq - 1]) if 1 <= kq <= pos.size else -1
        assert got[q] == want, (q, cc, kq)


@pytest.mark.parametrize("n,sigma", [(1, 1), (100, 1), (0, 4), (777, 2), (20000, 5), (300000, 256),
                                     (100000, 1 << 16), (50000, (1 << 20) + 7)])
def test_queries(wtmod, oracle_mod, n, sigma):
    rng = np.random.default_rng(n + 17)
    S = rng.integers(0, sigma, n).astype(inputs.dtype_for_sigma(sigma))
    say(f"[queries] n={n} sigma={sigma}")
    t = gpu_build(wtmod, S, sigma)
    _queries_check(wtmod, t, S, sigma, rng)


def test_queries_exhaustive_tiny(wtmod):
    rng = np.random.default_rng(5)
    for sigma in (2, 3, 5, 8):
        S = rng.integers(0, sigma, 40).astype(np.uint8)
        t = gpu_build(wtmod, S, sigma)
        n = S.size
        i = np.arange(n)
        assert np.array_equal(t.access(torch.from_numpy(i).cuda()).cpu().numpy(), S.astype(np.int32))
        cs, iis = np.meshgrid(np.arange(sigma + 2), np.arange(n + 1), indexing="ij")
        got = t.rank_query(torch.from_numpy(cs.ravel().astype(np.int32)).cuda(),
                           torch.from_numpy(iis.ravel()).cuda()).cpu().numpy()
        want = [pins.naive_rank(S, int(c), int(ii)) for c, ii in zip(cs.ravel(), iis.ravel())]
        assert list(got) == want
        cs, ks = np.meshgrid(np.arange(sigma + 2), np.arange(n + 2), indexing="ij")
        got = t.select_query(torch.from_numpy(cs.ravel().astype(np.int32)).cuda(),
                             torch.from_numpy(ks.ravel()).cuda()).cpu().numpy()
        want = [pins.naive_select(S, int(c), int(k)) if c < sigma else -1 for c, k in zip(cs.ravel(), ks.ravel())]
        assert list(got) == want


def test_lookback_fallback_forced(wtmod, oracle_mod):
    """Spin limit 0: every tile that finds a predecessor unpublished reduces it
    itself instead of waiting; outputs must not change."""
    wtmod.set_lookback_spin_limit(0)
    try:
        for cfg, n in [("text256", 1 << 21), ("alpha20", 1 << 19), ("uniform256", 1 << 20)]:
            S, sigma = inputs.workload(cfg, n)
            check_against_oracle(wtmod, oracle_mod, S, sigma, f"fallback {cfg} n={n}")
        S = np.random.default_rng(9).integers(0, 256, 300001).astype(np.uint8)
        t = gpu_build(wtmod, S, 256, directories=False)
        d = wtmod.build_rank_select(t.bits, S.size, t.L)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy().view(np.uint64) for k, v in d.items() if not k.startswith("_")}
        want = oracle_mod.rank_select(oracle_mod.build(S, 256)["bits"], S.size, t.L)
        assert_same(got, want, keys=("rank", "sel1", "sel0", "sel_counts"), ctx="fallback standalone")
    finally:
        wtmod.set_lookback_spin_limit(8)


def test_random_ragged_sweep(wtmod, oracle_mod):
    """Many short and ragged inputs (tails inside a 16-byte group, a row and
    a tile): every group past the end of a partial tile must leave the split
    untouched."""
    rng = np.random.default_rng(2024)
    cases = [(int(rng.integers(1, 300)), int(rng.choice([2, 5, 17, 256]))) for _ in range(120)]
    cases += [(int(rng.integers(16385, 16384 * 3)), int(rng.choice([4, 256]))) for _ in range(12)]
    cases += [(int(rng.integers(1, 9000)), int(rng.choice([300, 70000]))) for _ in range(12)]
    for n, sigma in cases:
        S = rng.integers(0, sigma, n, dtype=np.uint64).astype(inputs.dtype_for_sigma(sigma))
        t = gpu_build(wtmod, S, sigma)
        assert_same(t.to_numpy(), oracle_mod.build_all(S, sigma), ctx=f"sweep n={n} sigma={sigma}")


def test_query_multi_matches_single_tree_queries(wtmod):
    """wt_query_multi over several trees answers exactly what the one-tree
    kernels answer; a tree index out of range or an unknown kind gives
    WT_Q_BAD."""
    rng = np.random.default_rng(31)
    trees, seqs = [], []
    for n, sigma in [(1, 1), (5000, 3), (70000, 256), (20000, 1 << 16), (3000, (1 << 20) + 5), (0, 7)]:
        S = rng.integers(0, sigma, n).astype(inputs.dtype_for_sigma(sigma))
        trees.append(gpu_build(wtmod, S, sigma))
        seqs.append(S)
    views = wtmod.views_tensor(trees)
    m = 20000
    tix = rng.integers(0, len(trees) + 1, m)  # includes one bad index
    kind = rng.integers(0, 4, m)              # includes one bad kind
    a = np.zeros(m, np.int64)
    b = np.zeros(m, np.int64)
    for q in range(m):
        if tix[q] >= len(trees):
            continue
        S, n = seqs[tix[q]], seqs[tix[q]].size
        sig = trees[tix[q]].sigma
        if kind[q] == 0:
            a[q] = rng.integers(0, n + 2)
        else:
            a[q] = S[rng.integers(0, n)] if n and rng.random() < 0.8 else rng.integers(0, sig + 3)
            b[q] = rng.integers(0, n + 2) if kind[q] == 1 else rng.integers(0, 12)
    d = lambda x, dt: torch.from_numpy(x.astype(dt)).cuda()
    got = wtmod.query_multi(views, len(trees), d(tix, np.int32), d(kind, np.uint8), d(a, np.int64), d(b, np.int64))
    got = got.cpu().numpy()
    for ti, t in enumerate(trees):
        for kd in (0, 1, 2):
            sel = np.flatnonzero((tix == ti) & (kind == kd))
            if sel.size == 0:
                continue
            if kd == 0:
                want = t.access(d(a[sel], np.int64)).cpu().numpy().astype(np.int64) & 0xFFFFFFFF
            elif kd == 1:
                want = t.rank_query(d(a[sel], np.int32), d(b[sel], np.int64)).cpu().numpy()
            else:
                want = t.select_query(d(a[sel], np.int32), d(b[sel], np.int64)).cpu().numpy()
            assert np.array_equal(got[sel], want), (ti, kd)
    bad = (tix >= len(trees)) | (kind == 3)
    assert np.all(got[bad] == wtmod.Q_BAD)


def _expected_fused_level(C, sigma, L, half):
    """First level whose nodes all hold <= half positions, if <= L-2."""
    C = np.asarray(C, dtype=np.int64)
    for l in range(0, L - 1):
        ends = np.minimum(np.arange(0, (1 << l) + 1, dtype=np.int64) << (L - l), sigma)
        sizes = np.diff(C[ends])
        if sizes.max(initial=0) <= half:
            return l
    return L


@pytest.mark.parametrize("case", ["uniform_small", "uniform_mid", "uniform_deep", "sorted", "text", "u16",
                                  "u32", "ragged_nodes", "all_equal", "u32_narrow"])
def test_fused_levels_match_unfused(wtmod, oracle_mod, case):
    """Levels run fused in LDS give the same buffers as level passes, and
    fusion starts at the level the node sizes call for."""
    rng = np.random.default_rng(77)
    if case == "uniform_small":
        S, sigma = rng.integers(0, 256, 5000).astype(np.uint8), 256
    elif case == "uniform_mid":
        S, sigma = rng.integers(0, 256, 70001).astype(np.uint8), 256
    elif case == "uniform_deep":
        S, sigma = rng.integers(0, 200, 300017).astype(np.uint8), 200
    elif case == "sorted":
        S, sigma = np.sort(rng.integers(0, 256, 100000)).astype(np.uint8), 256
    elif case == "text":
        S, sigma = inputs.text_like(1 << 20), 256
    elif case == "u16":
        S, sigma = rng.integers(0, 1 << 16, 200000).astype(np.uint16), 1 << 16
    elif case == "u32":
        # 18 levels of 32-bit symbols whose dense tables (2^19 words) stay
        # small next to n: fused (a much larger alphabet takes the sparse
        # tables, which never fuse)
        S, sigma = rng.integers(0, (1 << 17) + 3, 150000).astype(np.uint32), (1 << 17) + 3
    elif case == "ragged_nodes":
        # node sizes of every magnitude: geometric symbol frequencies
        S = np.minimum(rng.geometric(0.02, 120000) - 1, 255).astype(np.uint8)
        S = rng.permutation(S)
        sigma = 256
    elif case == "all_equal":
        S, sigma = np.full(9000, 77, np.uint8), 128
    else:
        S, sigma = rng.integers(0, 60, 90000).astype(np.uint32), 60
    want = oracle_mod.build_all(S, sigma)
    L = want["L"]
    mid = 1 if L <= 8 else (2 if L <= 16 else 4)
    half = 16384 // mid // 2 - 32  # segment stride: the segment plus its offset in the first bit word fit 16 KiB
    l0 = _expected_fused_level(want["C"], sigma, L, half) if L >= 2 else L
    wtmod.set_fused_levels(True)
    t = gpu_build(wtmod, S, sigma)
    # The largest node of level l holds at least ceil(n / 2^l) positions;
    # when that rules out every level up to L-2 the build plans no fusion
    # (and leaves the plan word unwritten).
    lmin = next((l for l in range(64) if -(-S.size // (1 << l)) <= half), 64)
    if L >= 2 and lmin + 2 <= L:
        got_l0 = int(t.scratch[248:252].view(torch.int32).item())
    else:
        assert l0 == L, (case, l0, L, lmin)
        got_l0 = L
    assert got_l0 == l0, (case, got_l0, l0)
    assert_same(t.to_numpy(), want, ctx=f"{case} fused from level {l0} of {L}")
    wtmod.set_fused_levels(False)
    try:
        t2 = gpu_build(wtmod, S, sigma)
        assert_same(t2.to_numpy(), want, ctx=f"{case} unfused")
    finally:
        wtmod.set_fused_levels(True)
    if case in ("uniform_small", "uniform_mid", "u16", "u32", "sorted", "u32_narrow"):
        assert l0 < L - 1, (case, l0, L)  # these inputs exercise the fused path
