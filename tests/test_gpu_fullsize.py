"""Full-size checks: the text-like workload at n = 2^28 (the benchmark's
input and launch configuration) built as the binary tree, the wavelet
matrix, the 4-ary tree and the Huffman-shaped tree.
- The binary tree: every output buffer (bits, C, rank, sel1, sel0,
  sel_counts) equals the oracle's, bit for bit.
- The other shapes are checked against what holds at any size and against
  answers computed one by one: C against a numpy histogram of S; every
  level's popcount against the histogram (the count of symbols whose bit,
  resp. code bit, is set at that level), and the last rank entry; the
  Huffman code lengths and codes against the oracle's code construction on
  the same counts, and its level sizes against the weights; sampled access,
  rank and select answers against S itself.
- The sortWT construction (sorted copies of S, no level passes) against the
  level-pass build, every output buffer bit for bit.
Integer work: tolerance zero."""
import sys

import numpy as np
import pytest

from paper_1407_8142_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

POPC8 = np.array([bin(x).count("1") for x in range(256)], dtype=np.int64)


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


@pytest.fixture(scope="module")
def text(wtmod):
    say("[fullsize] generating text-like n=2^28")
    S, sigma = inputs.workload("text256")
    hist = np.bincount(S, minlength=sigma).astype(np.int64)
    return S, sigma, hist, wtmod.to_device(S)


def popcounts(words: torch.Tensor) -> np.ndarray:
    """Popcount of each row of an int64 tensor of bit words."""
    b = words.contiguous().cpu().numpy().view(np.uint8).reshape(words.shape[0], -1)
    return POPC8[b].sum(axis=1)


def sampled_queries(S, access, rank_query, select_query, seed):
    rng = np.random.default_rng(seed)
    n = S.size
    dev = torch.device("cuda")
    i = rng.integers(0, n, 4000)
    acc = access(torch.from_numpy(i).to(dev)).cpu().numpy()
    assert np.array_equal(acc.astype(np.int64), S[i].astype(np.int64))
    cs = S[rng.integers(0, n, 12)].astype(np.int64)
    js = rng.integers(0, n + 1, 12)
    rk = rank_query(torch.from_numpy(cs).to(dev), torch.from_numpy(js).to(dev)).cpu().numpy()
    for c, j, r in zip(cs, js, rk):
        assert int(r) == int(np.count_nonzero(S[:j] == c)), (c, j)
    ks = []
    for c in cs:
        pos = np.flatnonzero(S == c)
        k = int(rng.integers(1, pos.size + 1))
        ks.append((k, int(pos[k - 1])))
    sl = select_query(torch.from_numpy(cs).to(dev),
                      torch.tensor([k for k, _ in ks], dtype=torch.int64, device=dev)).cpu().numpy()
    assert [int(x) for x in sl] == [p for _, p in ks]


def C_of(hist):
    return np.concatenate([[0], np.cumsum(hist)]).astype(np.uint64)


def test_fullsize_tree(wtmod, oracle_mod, text):
    S, sigma, hist, d = text
    L = 8
    say("[fullsize] binary tree")
    t = wtmod.build(d, sigma)
    torch.cuda.synchronize()
    assert t.status() == wtmod.WT_OK
    assert np.array_equal(t.C.cpu().numpy().view(np.uint64), C_of(hist))
    pc = popcounts(t.bits)
    for l in range(L):
        ones = int(sum(hist[c] for c in range(sigma) if (c >> (L - 1 - l)) & 1))
        assert int(pc[l]) == ones, l
        assert int(t.rank[l, -1].item()) == ones
    sampled_queries(S, t.access, t.rank_query, t.select_query, 1)
    got = t.to_numpy()
    del t
    torch.cuda.empty_cache()
    say("[fullsize] binary tree against the oracle")
    want = oracle_mod.build_all(S, sigma)
    for k in ("bits", "C", "rank", "sel1", "sel0", "sel_counts"):
        g = np.asarray(got[k], dtype=np.uint64).reshape(-1)
        w = np.asarray(want[k], dtype=np.uint64).reshape(-1)
        assert g.shape == w.shape, k
        bad = np.flatnonzero(g != w)
        assert bad.size == 0, f"{k} differs at {bad.size} entries, first {bad[:5]}"


def test_fullsize_matrix(wtmod, text):
    S, sigma, hist, d = text
    L = 8
    say("[fullsize] wavelet matrix")
    m = wtmod.build_matrix(d, sigma)
    torch.cuda.synchronize()
    assert m.status() == wtmod.WT_OK
    got = m.to_numpy()
    assert np.array_equal(got["C"], C_of(hist))
    pc = popcounts(m.tree.bits)
    for l in range(L):
        ones = int(sum(hist[c] for c in range(sigma) if (c >> (L - 1 - l)) & 1))
        assert int(pc[l]) == ones and int(got["zeros"][l]) == S.size - ones, l
    sampled_queries(S, m.access, m.rank_query, m.select_query, 2)
    del m
    torch.cuda.empty_cache()


def test_fullsize_multiary(wtmod, text):
    S, sigma, hist, d = text
    say("[fullsize] 4-ary tree")
    t = wtmod.build_multiary(d, sigma)
    torch.cuda.synchronize()
    assert t.status() == wtmod.WT_OK
    assert np.array_equal(t.C.cpu().numpy().view(np.uint64), C_of(hist))
    sampled_queries(S, t.access, t.rank_query, t.select_query, 3)
    del t
    torch.cuda.empty_cache()


def test_fullsize_huffman(wtmod, oracle_mod, text):
    S, sigma, hist, d = text
    say("[fullsize] Huffman-shaped tree")
    t = wtmod.build_huffman(d, sigma)
    torch.cuda.synchronize()
    assert t.status() == wtmod.WT_OK
    got = t.to_numpy()
    lens, h = oracle_mod.huffman_lengths(hist.astype(np.uint64))
    codes = oracle_mod.huffman_codes(lens)
    assert got["h"] == h
    assert np.array_equal(got["lens"][:sigma], lens) and np.array_equal(got["codes"][:sigma], codes)
    assert np.array_equal(got["C"], C_of(hist))
    pc = popcounts(t.bits[:h])
    for dd in range(h):
        deeper = [c for c in range(sigma) if hist[c] and lens[c] > dd]
        assert int(got["nd"][dd]) == int(sum(hist[c] for c in deeper)), dd
        ones = int(sum(hist[c] for c in deeper if (int(codes[c]) >> (63 - dd)) & 1))
        assert int(pc[dd]) == ones and int(got["rank"][dd, -1]) == ones, dd
    sampled_queries(S, t.access, t.rank_query, t.select_query, 4)
    del t
    torch.cuda.empty_cache()


def test_fullsize_sort_equals_level_passes(wtmod, text):
    S, sigma, hist, d = text
    say("[fullsize] sortWT against the level passes")
    a = wtmod.build(d, sigma)
    b = wtmod.build_sort(d, sigma)
    torch.cuda.synchronize()
    assert a.status() == wtmod.WT_OK and b.status() == wtmod.WT_OK
    for k in ("bits", "C", "rank", "sel1", "sel0", "sel_counts"):
        assert torch.equal(getattr(a, k), getattr(b, k)), k
    del a, b
    torch.cuda.empty_cache()
