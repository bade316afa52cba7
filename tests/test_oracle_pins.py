"""CPU tests that pin the oracle to facts other than itself (no GPU needed)."""
import itertools
import json
import os

import numpy as np
import pytest

import pins
from oracle import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "handworked.json")


def _tree_with_dirs(S, sigma, lib_path=oracle.LIB):
    return oracle.build_all(np.asarray(S), sigma, lib_path)


def _dtype(sigma):
    return np.uint8 if sigma <= 256 else (np.uint16 if sigma <= 65536 else np.uint32)


def query_failures(t, S, sigma, lib_path=oracle.LIB):
    """Exhaustive tree-walk queries against naive counting over S."""
    n = S.shape[0]
    for i in range(n):
        if oracle.access_tree(t, i, lib_path) != int(S[i]):
            return ["access_tree"]
    for c in range(sigma + 1):
        for i in range(n + 1):
            if oracle.rank_tree(t, c, i, lib_path) != pins.naive_rank(S, c, i):
                return ["rank_tree"]
        if c < sigma:
            for k in range(n + 2):
                if oracle.select_tree(t, c, k, lib_path) != pins.naive_select(S, c, k):
                    return ["select_tree"]
    return []


def test_golden_handworked():
    doc = json.load(open(GOLDEN))
    for case in doc["cases"]:
        sigma = case["sigma"]
        S = np.asarray(case["S"], dtype=_dtype(sigma))
        t = _tree_with_dirs(S, sigma)
        assert t["L"] == len(case["levels"]), case["name"]
        for l, row in enumerate(case["levels"]):
            assert list(pins.unpack(t["bits"][l], len(S))) == row, (case["name"], l)
            assert [int(w) for w in t["bits"][l]] == case["words"][l], (case["name"], l)
        assert [int(x) for x in t["C"]] == case["C"], case["name"]
        for c, i, want in case["rank"]:
            assert oracle.rank_tree(t, c, i) == want, (case["name"], c, i)
            assert oracle.rank_naive(S, c, i) == want
        for c, k, want in case["select"]:
            assert oracle.select_tree(t, c, k) == want, (case["name"], c, k)
            assert oracle.select_naive(S, c, k) == want
        for i, s in enumerate(case["S"]):
            assert oracle.access_tree(t, i) == s


@pytest.mark.parametrize("sigma", [1, 2, 3, 4, 5])
def test_exhaustive_tiny(sigma):
    """Every sequence of length <= 5 (<= 4 for the query sweep) over [0, sigma)."""
    for n in range(0, 6):
        for tup in itertools.product(range(sigma), repeat=n):
            S = np.asarray(tup, dtype=np.uint8)
            t = _tree_with_dirs(S, sigma)
            exp = pins.sortwt_levels_py(list(tup), sigma)
            fails = pins.check_tree(t, S, sigma, exp)
            assert not fails, (tup, fails)
            if n <= 4:
                assert not query_failures(t, S, sigma), tup


@pytest.mark.parametrize("sigma", [6, 7, 8, 9, 16, 17])
def test_exhaustive_short_wider_alphabets(sigma):
    for n in range(0, 4):
        for tup in itertools.product(range(sigma), repeat=n):
            S = np.asarray(tup, dtype=np.uint8)
            t = _tree_with_dirs(S, sigma)
            assert not pins.check_tree(t, S, sigma, pins.sortwt_levels_py(list(tup), sigma)), tup


@pytest.mark.parametrize("n,sigma,seed", [
    (1000, 3, 1), (4095, 146, 2), (4097, 256, 3), (10000, 256, 4), (513, 1 << 16, 5),
    (10000, 1 << 16, 6), (9000, (1 << 20) - 3, 7), (8193, 1 << 20, 8), (20000, 5, 9), (70000, 2, 10),
])
def test_random_medium(n, sigma, seed):
    rng = np.random.default_rng(seed)
    S = rng.integers(0, sigma, n).astype(_dtype(sigma))
    t = _tree_with_dirs(S, sigma)
    assert not pins.check_tree(t, S, sigma)


def test_random_medium_skewed_and_queries():
    rng = np.random.default_rng(11)
    sigma = 200
    S = np.minimum(rng.zipf(1.3, 3000) - 1, sigma - 1).astype(np.uint8)
    t = _tree_with_dirs(S, sigma)
    assert not pins.check_tree(t, S, sigma)
    for i in rng.integers(0, S.size, 50):
        assert oracle.access_tree(t, int(i)) == int(S[i])
    for _ in range(50):
        c, i = int(rng.integers(0, sigma + 3)), int(rng.integers(0, S.size + 2))
        assert oracle.rank_tree(t, c, i) == pins.naive_rank(S, c, i)
        k = int(rng.integers(0, 40))
        if c < sigma:
            assert oracle.select_tree(t, c, k) == pins.naive_select(S, c, k)


def test_special_cases():
    rng = np.random.default_rng(12)
    # sigma = 2: B_0 is S itself.
    S = rng.integers(0, 2, 777).astype(np.uint8)
    t = oracle.build(S, 2)
    assert np.array_equal(pins.unpack(t["bits"][0], S.size), S)
    # Constant input c: every level is the constant bit of c.
    for c, sigma in [(0, 256), (255, 256), (77, 100), (4, 5)]:
        S = np.full(1000, c, dtype=np.uint8)
        t = oracle.build(S, sigma)
        L = pins.levels(sigma)
        for l in range(L):
            assert set(pins.unpack(t["bits"][l], S.size)) == {(c >> (L - 1 - l)) & 1}
    # Sorted input: every S_l equals S, so B_l[i] is bit L-1-l of S[i].
    S = np.sort(rng.integers(0, 1000, 3000)).astype(np.uint16)
    t = oracle.build(S, 1000)
    for l in range(t["L"]):
        assert np.array_equal(pins.unpack(t["bits"][l], S.size), (S >> (t["L"] - 1 - l)) & 1)
    # sigma = 1: no levels at all.
    t = oracle.build(np.zeros(10, dtype=np.uint8), 1)
    assert t["L"] == 0 and t["bits"].size == 0 and list(t["C"]) == [0, 10]
    # n = 0.
    t = oracle.build_all(np.zeros(0, dtype=np.uint8), 256)
    assert t["bits"].size == 0 and not t["C"].any()
    assert t["rank"].shape == (8, 1) and not t["rank"].any()
    assert t["sel1"].shape == (8, 1) and not t["sel1"].any() and not t["sel_counts"].any()


def test_levels_integer():
    assert [pins.levels(s) for s in (1, 2, 3, 4, 5, 255, 256, 257)] == [0, 1, 2, 2, 3, 8, 8, 9]
    for s in (1, 2, 3, 4, 5, 255, 256, 257, (1 << 20) - 1, 1 << 20, (1 << 20) + 1, 1 << 31, (1 << 31) + 1,
              1 << 32):
        assert oracle.levels(s) == pins.levels(s)


def test_error_paths():
    with pytest.raises(oracle.OracleError):
        oracle.build(np.asarray([0, 1, 5], dtype=np.uint8), 5)
    with pytest.raises(oracle.OracleError):
        oracle.build(np.asarray([0], dtype=np.uint8), 0)
    with pytest.raises(oracle.OracleError):
        oracle.build(np.asarray([0], dtype=np.uint8), 257)


def _pin_failures(lib_path):
    """Run every pin on a few inputs through the oracle built at lib_path."""
    fails = set()
    rng = np.random.default_rng(13)
    cases = [(np.asarray(c, dtype=np.uint8), s) for c, s in [
        ([3, 1, 0, 2, 3, 0, 1, 2], 4), ([4, 0, 3, 1, 4, 2], 5)]]
    cases.append((rng.integers(0, 256, 5000).astype(np.uint8), 256))
    cases.append((rng.integers(0, 13, 700).astype(np.uint8), 13))
    for S, sigma in cases:
        try:
            t = _tree_with_dirs(S, sigma, lib_path)
        except oracle.OracleError:
            fails.add("error")
            continue
        fails.update(pins.check_tree(t, S, sigma))
        if S.size <= 8:
            fails.update(query_failures(t, S, sigma, lib_path))
    return fails


def test_pins_catch_planted_mutants(tmp_path):
    assert _pin_failures(oracle.LIB) == set()
    for m in (1, 2, 3, 4, 5):
        path = str(tmp_path / f"liboracle_m{m}.so")
        oracle.compile_oracle(path, mutant=m)
        assert _pin_failures(path), f"mutant {m} passed every pin"


# ---- wavelet matrix -----------------------------------------------------------

def matrix_query_failures(t, S, sigma, lib_path=oracle.LIB):
    """Exhaustive matrix-walking queries against naive counting over S."""
    n = S.shape[0]
    for i in range(n):
        if oracle.access_matrix(t, i, lib_path) != int(S[i]):
            return ["access_matrix"]
    for c in range(sigma + 1):
        for i in range(n + 1):
            if oracle.rank_matrix(t, c, i, lib_path) != pins.naive_rank(S, c, i):
                return ["rank_matrix"]
        for k in range(n + 2):
            if oracle.select_matrix(t, c, k, lib_path) != pins.naive_select(S, c, k):
                return ["select_matrix"]
    return []


@pytest.mark.parametrize("sigma", [1, 2, 3, 4, 5])
def test_matrix_exhaustive_tiny(sigma):
    """Every sequence of length <= 4 (<= 5 for sigma <= 3): the sort view,
    the zero counts, the directories and every query."""
    for n in range(0, 6 if sigma <= 3 else 5):
        for seq in itertools.product(range(sigma), repeat=n):
            S = np.asarray(seq, dtype=np.uint8)
            t = oracle.build_matrix_all(S, sigma)
            assert pins.check_matrix(t, S, sigma) == [], (seq, sigma)
            assert matrix_query_failures(t, S, sigma) == [], (seq, sigma)


@pytest.mark.parametrize("sigma", [6, 7, 8, 9, 16, 17])
def test_matrix_exhaustive_short_wider(sigma):
    for n in range(0, 4):
        for seq in itertools.product(range(sigma), repeat=n):
            S = np.asarray(seq, dtype=np.uint8)
            t = oracle.build_matrix_all(S, sigma)
            assert pins.check_matrix(t, S, sigma) == [], (seq, sigma)
            assert matrix_query_failures(t, S, sigma) == [], (seq, sigma)


@pytest.mark.parametrize("n,sigma,seed", [(1000, 256, 1), (70000, 256, 2), (33333, 5, 3), (20000, 1 << 16, 4),
                                          (9000, (1 << 20) + 7, 5), (4097, 300, 6)])
def test_matrix_random_medium(n, sigma, seed):
    rng = np.random.default_rng(seed)
    S = rng.integers(0, sigma, n).astype(_dtype(sigma))
    t = oracle.build_matrix_all(S, sigma)
    assert pins.check_matrix(t, S, sigma) == []
    for _ in range(40):
        i = int(rng.integers(0, n))
        assert oracle.access_matrix(t, i) == int(S[i])
        c = int(S[int(rng.integers(0, n))])
        j = int(rng.integers(0, n + 1))
        assert oracle.rank_matrix(t, c, j) == pins.naive_rank(S, c, j)
        k = int(rng.integers(1, pins.naive_rank(S, c, n) + 2))
        assert oracle.select_matrix(t, c, k) == pins.naive_select(S, c, k)


def test_matrix_equals_tree_for_binary_alphabets():
    """With one level (sigma = 2) the matrix and the tree hold the same bits;
    sigma = 1 has no levels at all."""
    rng = np.random.default_rng(21)
    for n in (0, 1, 63, 64, 65, 5000):
        S = rng.integers(0, 2, n).astype(np.uint8)
        m, tr = oracle.build_matrix(S, 2), oracle.build(S, 2)
        assert np.array_equal(m["bits"], tr["bits"])
        assert int(m["zeros"][0]) == int(n - S.sum())
        m1 = oracle.build_matrix(np.zeros(n, np.uint8), 1)
        assert m1["L"] == 0 and m1["bits"].size == 0


def test_matrix_rejects_symbols():
    with pytest.raises(oracle.OracleError):
        oracle.build_matrix(np.asarray([0, 5], dtype=np.uint8), 5)


def _matrix_pin_failures(lib_path):
    fails = set()
    rng = np.random.default_rng(14)
    cases = [(np.asarray(c, dtype=np.uint8), s) for c, s in [([3, 1, 0, 2, 3, 0, 1, 2], 4), ([4, 0, 3, 1, 4, 2], 5)]]
    cases.append((rng.integers(0, 256, 5000).astype(np.uint8), 256))
    for S, sigma in cases:
        t = oracle.build_matrix_all(S, sigma, lib_path)
        fails.update(pins.check_matrix(t, S, sigma))
        if S.size <= 8:
            fails.update(matrix_query_failures(t, S, sigma, lib_path))
    return fails


def test_matrix_pins_catch_planted_mutants(tmp_path):
    assert _matrix_pin_failures(oracle.LIB) == set()
    for m in (6, 7):
        path = str(tmp_path / f"liboracle_m{m}.so")
        oracle.compile_oracle(path, mutant=m)
        assert _matrix_pin_failures(path), f"mutant {m} passed every matrix pin"


# ---- multiary wavelet tree (d = 4) --------------------------------------------

def multiary_query_failures(t, S, sigma, lib_path=oracle.LIB):
    n = S.shape[0]
    for i in range(n):
        if oracle.access_multiary(t, i, lib_path) != int(S[i]):
            return ["access_multiary"]
    for c in range(sigma + 1):
        for i in range(n + 1):
            if oracle.rank_multiary(t, c, i, lib_path) != pins.naive_rank(S, c, i):
                return ["rank_multiary"]
        for k in range(n + 2):
            want = pins.naive_select(S, c, k) if c < sigma else -1
            if oracle.select_multiary(t, c, k, lib_path) != want:
                return ["select_multiary"]
    return []


@pytest.mark.parametrize("sigma", [1, 2, 3, 4, 5, 8])
def test_multiary_exhaustive_tiny(sigma):
    for n in range(0, 5 if sigma <= 5 else 4):
        for seq in itertools.product(range(sigma), repeat=n):
            S = np.asarray(seq, dtype=np.uint8)
            t = oracle.build_multiary_all(S, sigma)
            assert pins.check_multiary(t, S, sigma) == [], (seq, sigma)
            assert multiary_query_failures(t, S, sigma) == [], (seq, sigma)


@pytest.mark.parametrize("n,sigma,seed", [(1000, 256, 1), (70000, 256, 2), (33333, 5, 3), (20000, 1 << 16, 4),
                                          (9000, (1 << 20) + 7, 5), (4097, 300, 6), (5000, 128, 7)])
def test_multiary_random_medium(n, sigma, seed):
    rng = np.random.default_rng(seed)
    S = rng.integers(0, sigma, n).astype(_dtype(sigma))
    t = oracle.build_multiary_all(S, sigma)
    assert pins.check_multiary(t, S, sigma) == []
    for _ in range(30):
        i = int(rng.integers(0, n))
        assert oracle.access_multiary(t, i) == int(S[i])
        c = int(S[int(rng.integers(0, n))])
        j = int(rng.integers(0, n + 1))
        assert oracle.rank_multiary(t, c, j) == pins.naive_rank(S, c, j)
        k = int(rng.integers(1, pins.naive_rank(S, c, n) + 2))
        assert oracle.select_multiary(t, c, k) == pins.naive_select(S, c, k)


def test_multiary_relates_to_binary_tree():
    """With an even number of binary levels, the high bit of every entry of
    4-ary level j is binary level 2j's bit at the same position (both levels
    list S sorted by its top 2j bits); for sigma <= 4 the one level is S."""
    rng = np.random.default_rng(31)
    for sigma in (4, 16, 256, 1 << 12):
        S = rng.integers(0, sigma, 3001).astype(_dtype(sigma))
        m, tr = oracle.build_multiary(S, sigma), oracle.build(S, sigma)
        for j in range(m["Lq"]):
            row = pins.unpack(m["digits"][j].view(np.uint8).view(np.uint64), 2 * S.size)
            hi = row[1::2]
            assert np.array_equal(hi, pins.unpack(tr["bits"][2 * j], S.size)), (sigma, j)
    S = rng.integers(0, 4, 777).astype(np.uint8)
    assert np.array_equal(oracle.build_multiary(S, 4)["digits"][0], pins.pack4(S, S.size))


def test_multiary_pins_catch_planted_mutant(tmp_path):
    def failures(path):
        f = set()
        rng = np.random.default_rng(15)
        for S, sigma in [(np.asarray([3, 1, 0, 2, 3, 0, 1, 2, 5, 7], np.uint8), 8),
                         (rng.integers(0, 256, 4000).astype(np.uint8), 256)]:
            t = oracle.build_multiary_all(S, sigma, path)
            f.update(pins.check_multiary(t, S, sigma))
        return f
    assert failures(oracle.LIB) == set()
    path = str(tmp_path / "liboracle_m8.so")
    oracle.compile_oracle(path, mutant=8)
    assert failures(path), "mutant 8 passed every multiary pin"
