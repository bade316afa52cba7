"""Pins of the oracle's Huffman-shaped wavelet tree (section "Extensions";
readings listed in oracle/wt_oracle.c).  None of these re-types the oracle:
- hand-derived code lengths for tie-breaking cases (the merge order is
  (weight, leaves first, symbol / creation order));
- optimality: on tiny alphabets the oracle's cost sum(w * len) equals the
  minimum over every length vector with Kraft sum 1 (brute force);
- canonical codes: prefix-free, Kraft sum 1, increasing in (length, symbol);
- an independent decoder that walks the level bitmaps back to S (pins the
  node order and the stability of every level);
- level sizes and popcounts from the weights and codes;
- equal weights over a power-of-two alphabet reduce to the binary tree of
  the levelWT oracle;
- a planted mutant (internal nodes first on ties) fails the tie fixtures."""
import itertools

import numpy as np
import pytest

from oracle import oracle


def unpack(words: np.ndarray, m: int) -> np.ndarray:
    b = np.unpackbits(np.ascontiguousarray(words, dtype="<u8").view(np.uint8), bitorder="little")
    return b[:m].astype(np.int64)


# Tie fixtures, derived by hand from the merge order:
#  (1,1,2,2): s0+s1 -> A(2); then s2(2, leaf) and s3(2, leaf) come before A(2)
#             -> B(4); then A+B: every length 2.
#  (5,1,1,2): s1+s2 -> A(2); s3(2, leaf) before A(2) -> s3+A = B(4); B+s0.
#             lengths s0 1, s1 3, s2 3, s3 2.
#  (1,1,1):   s0+s1 -> A(2); s2+A: lengths 2, 2, 1.
#  (3,0,3):   absent symbol 1 has no leaf; two leaves of length 1.
TIES = [((1, 1, 2, 2), (2, 2, 2, 2)), ((5, 1, 1, 2), (1, 3, 3, 2)), ((1, 1, 1), (2, 2, 1)), ((3, 0, 3), (1, 0, 1))]


@pytest.mark.parametrize("w,want", TIES)
def test_tie_fixtures(w, want):
    lens, h = oracle.huffman_lengths(np.array(w))
    assert tuple(int(x) for x in lens) == want
    assert h == max(want)


def test_mutant_internal_first_fails(tmp_path):
    path = str(tmp_path / "liboracle_m9.so")
    oracle.compile_oracle(path, mutant=9)
    got = [tuple(int(x) for x in oracle.huffman_lengths(np.array(w), lib_path=path)[0]) for w, _ in TIES]
    assert any(g != want for g, (_, want) in zip(got, TIES))


def kraft_vectors(k: int, lmax: int):
    for ls in itertools.product(range(1, lmax + 1), repeat=k):
        if sum(2.0 ** -x for x in ls) == 1.0:
            yield ls


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6])
def test_optimal_cost_brute_force(k):
    rng = np.random.default_rng(100 + k)
    vecs = list(kraft_vectors(k, k - 1))
    for _ in range(20):
        w = rng.integers(1, 30, k)
        lens, _ = oracle.huffman_lengths(w)
        best = min(sum(int(a) * b for a, b in zip(w, ls)) for ls in vecs)
        assert sum(int(a) * int(b) for a, b in zip(w, lens)) == best


@pytest.mark.parametrize("seed", range(6))
def test_canonical_codes(seed):
    rng = np.random.default_rng(seed)
    sigma = int(rng.integers(2, 257))
    w = rng.geometric(0.05, sigma) * (rng.random(sigma) < 0.8)
    lens, h = oracle.huffman_lengths(w)
    codes = oracle.huffman_codes(lens)
    present = [c for c in range(sigma) if w[c]]
    if len(present) < 2:
        return
    assert sum(2.0 ** -int(lens[c]) for c in present) == 1.0
    strs = {c: format(int(codes[c]) >> (64 - int(lens[c])), f"0{int(lens[c])}b") for c in present}
    for a in present:
        for b in present:
            if a != b:
                assert not strs[b].startswith(strs[a])
    order = sorted(present, key=lambda c: (int(lens[c]), c))
    assert all(int(codes[x]) < int(codes[y]) for x, y in zip(order, order[1:]))
    assert h == max(int(lens[c]) for c in present)


def decode_all(t: dict, S: np.ndarray) -> np.ndarray:
    """Walks every position down the levels, using only the weights, the
    codes and the bitmaps: the node of a position at depth d is the code
    prefix read so far, its start in level d is the weight of the symbols
    with a longer code and a smaller prefix, and a child's position is its
    start plus the rank of the bit inside the node."""
    lens, codes, w = t["lens"], t["codes"], t["weights"]
    sym_of = {(int(lens[c]), int(codes[c]) >> (64 - int(lens[c]))): c for c in range(len(lens)) if w[c] and lens[c]}
    B = [unpack(t["bits"][d], int(t["nd"][d])) for d in range(t["h"])]

    def start(d: int, p: int) -> int:
        return int(sum(int(w[c]) for c in range(len(lens))
                       if w[c] and lens[c] > d and (int(codes[c]) >> (64 - d) if d else 0) < p))

    out = np.zeros(S.size, dtype=np.int64)
    if t["h"] == 0:
        present = [c for c in range(len(lens)) if w[c]]
        out[:] = present[0] if present else 0
        return out
    for i in range(S.size):
        pos, p = i, 0
        for d in range(t["h"]):
            s = start(d, p)
            b = int(B[d][pos])
            inside = B[d][s:pos]
            r = int(inside.sum()) if b else int(inside.size - inside.sum())
            p = (p << 1) | b
            if (d + 1, p) in sym_of:
                out[i] = sym_of[(d + 1, p)]
                break
            pos = start(d + 1, p) + r
    return out


@pytest.mark.parametrize("case", ["hand", "zipf", "uniform", "two", "one", "empty", "skewed"])
def test_decode_and_sizes(case):
    rng = np.random.default_rng(7)
    if case == "hand":
        S, sigma = np.array([0, 3, 1, 0, 2, 0, 0, 3, 0], np.uint8), 4
    elif case == "zipf":
        ranks = np.minimum(rng.zipf(1.3, 3000), 40) - 1
        S, sigma = ranks.astype(np.uint8), 40
    elif case == "uniform":
        S, sigma = rng.integers(0, 13, 2000).astype(np.uint8), 13
    elif case == "two":
        S, sigma = rng.integers(0, 2, 500).astype(np.uint8) * 7, 9
    elif case == "one":
        S, sigma = np.full(300, 5, np.uint8), 6
    elif case == "empty":
        S, sigma = np.zeros(0, np.uint8), 5
    else:  # Fibonacci-like weights: a deep, thin tree
        fib = [1, 1]
        while len(fib) < 14:
            fib.append(fib[-1] + fib[-2])
        S = np.repeat(np.arange(14), fib).astype(np.uint8)
        S, sigma = rng.permutation(S), 14
    t = oracle.build_huffman(S, sigma)
    assert np.array_equal(decode_all(t, S), S.astype(np.int64))
    lens, codes, w = t["lens"], t["codes"], t["weights"]
    for d in range(t["h"]):
        deeper = [c for c in range(sigma) if w[c] and lens[c] > d]
        assert int(t["nd"][d]) == sum(int(w[c]) for c in deeper)
        ones = sum(int(w[c]) for c in deeper if (int(codes[c]) >> (63 - d)) & 1)
        assert int(unpack(t["bits"][d], int(t["nd"][d])).sum()) == ones
        tail = unpack(t["bits"][d], t["W"] * 64)[int(t["nd"][d]):]
        assert not tail.any()
    assert int(t["nd"].sum()) == sum(int(w[c]) * int(lens[c]) for c in range(sigma))
    if case == "skewed":
        assert t["h"] == 13


@pytest.mark.parametrize("L", [1, 2, 3, 8])
def test_equal_weights_reduce_to_the_binary_tree(L):
    sigma = 1 << L
    rng = np.random.default_rng(L)
    S = rng.permutation(np.repeat(np.arange(sigma), 3)).astype(np.uint8)
    t = oracle.build_huffman(S, sigma)
    assert t["h"] == L and (t["lens"] == L).all()
    b = oracle.build(S, sigma)
    assert np.array_equal(t["bits"], b["bits"])


def test_directories_naive():
    rng = np.random.default_rng(3)
    S = (np.minimum(rng.zipf(1.2, 70000), 200) - 1).astype(np.uint8)
    t = oracle.build_huffman_all(S, 200)
    n = S.size
    for d in range(t["h"]):
        m = int(t["nd"][d])
        B = unpack(t["bits"][d], m)
        cs = np.concatenate([[0], np.cumsum(B)])
        for j in range(t["rank"].shape[1]):
            assert int(t["rank"][d, j]) == int(cs[min(512 * j, m)])
        ones, zeros = np.flatnonzero(B == 1), np.flatnonzero(B == 0)
        s1, s0 = ones[::4096], zeros[::4096]
        assert np.array_equal(t["sel1"][d, : s1.size], s1) and (t["sel1"][d, s1.size:] == m).all()
        assert np.array_equal(t["sel0"][d, : s0.size], s0) and (t["sel0"][d, s0.size:] == m).all()
        assert int(t["sel_counts"][d]) == s1.size and int(t["sel_counts"][t["h"] + d]) == s0.size
    assert t["rank"].shape[1] == (n + 511) // 512 + 1
