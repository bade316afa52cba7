"""Independent checks ("pins") for wavelet-tree outputs, in plain Python/numpy.

None of these re-types the oracle: each one states a different fact that the
paper or the mathematics fixes.

  sortwt_levels   Fig. 2 (sortWT): level l is S stably sorted by its top l
                  bits, and B_l holds bit L-1-l of that order.
  popcount        ones on level l = number of symbols with bit L-1-l set.
  histogram       C[c] = #{i : S[i] < c} by numpy bincount/cumsum.
  node offsets    Fig. 1 child rule: the right child of node p starts where
                  the left child's zeros end.
  directories     rank/select samples by a cumulative count over the bits.
  queries         naive counting over S.
  matrix levels   the wavelet matrix's sort view (the paper's extensions):
                  level l lists S stably sorted by the reverse of its top l
                  bits, and its bitmap holds bit L-1-l of that order.
  matrix zeros    the zeros of matrix level l = number of symbols whose bit
                  L-1-l is 0.
  4-ary levels    the multiary tree (d = 4) in the sortWT view: level j lists
                  S stably sorted by its top j base-4 digits, and its entry
                  is digit j; the digit counts of a level are those of S.
"""
from __future__ import annotations

import numpy as np

RANK_BLOCK_BITS = 512
SEL_SAMPLE = 4096


def levels(sigma: int) -> int:
    return (sigma - 1).bit_length() if sigma > 1 else 0


def pack(bitrow, n: int) -> np.ndarray:
    """LSB-first packing of a 0/1 sequence of length n into ceil(n/64) words."""
    W = (n + 63) // 64
    b = np.zeros(W * 64, dtype=np.uint8)
    b[:n] = np.asarray(bitrow, dtype=np.uint8)[:n]
    return np.packbits(b.reshape(-1, 8), axis=1, bitorder="little").reshape(-1).view(np.uint64) \
        if W else np.zeros(0, dtype=np.uint64)


def unpack(words: np.ndarray, n: int) -> np.ndarray:
    if n == 0:
        return np.zeros(0, dtype=np.uint8)
    return np.unpackbits(np.ascontiguousarray(words, dtype=np.uint64).view(np.uint8),
                         bitorder="little")[:n]


def sortwt_levels_py(S, sigma: int):
    """Pure-Python stable ``sorted`` per level (tiny inputs)."""
    L = levels(sigma)
    out = []
    for l in range(L):
        k = L - 1 - l
        T = sorted(S, key=lambda s: s >> (k + 1))
        out.append([(s >> k) & 1 for s in T])
    return out


def sortwt_levels_np(S: np.ndarray, sigma: int) -> list[np.ndarray]:
    """numpy stable argsort per level (medium inputs)."""
    L = levels(sigma)
    S64 = S.astype(np.uint64)
    out = []
    for l in range(L):
        k = L - 1 - l
        order = np.argsort(S64 >> np.uint64(k + 1), kind="stable")
        out.append(((S64[order] >> np.uint64(k)) & np.uint64(1)).astype(np.uint8))
    return out


def expected_C(S: np.ndarray, sigma: int) -> np.ndarray:
    cnt = np.bincount(S.astype(np.int64), minlength=sigma)[:sigma].astype(np.uint64)
    return np.concatenate([[np.uint64(0)], np.cumsum(cnt, dtype=np.uint64)])


def naive_dirs(bits_rows: list[np.ndarray], n: int) -> dict:
    L = len(bits_rows)
    rank_len = (n + RANK_BLOCK_BITS - 1) // RANK_BLOCK_BITS + 1
    cap = (n + SEL_SAMPLE - 1) // SEL_SAMPLE + 1
    rank = np.zeros((L, rank_len), dtype=np.uint64)
    sel1 = np.full((L, cap), n, dtype=np.uint64)
    sel0 = np.full((L, cap), n, dtype=np.uint64)
    counts = np.zeros(2 * L, dtype=np.uint64)
    for l, b in enumerate(bits_rows):
        b = np.asarray(b, dtype=np.int64)
        cs = np.concatenate([[0], np.cumsum(b)])
        pos = np.minimum(np.arange(rank_len, dtype=np.int64) * RANK_BLOCK_BITS, n)
        rank[l] = cs[pos]
        ones = np.flatnonzero(b == 1)
        zeros = np.flatnonzero(b == 0)
        s1 = ones[::SEL_SAMPLE]
        s0 = zeros[::SEL_SAMPLE]
        sel1[l, : s1.size] = s1
        sel0[l, : s0.size] = s0
        counts[l] = s1.size
        counts[L + l] = s0.size
    return {"rank": rank, "sel1": sel1, "sel0": sel0, "sel_counts": counts}


def check_tree(t: dict, S: np.ndarray, sigma: int, expected_levels=None) -> list[str]:
    """Return the names of the pins that the built tree ``t`` ({'bits','C',...}) fails."""
    fails = []
    n = S.shape[0]
    L = levels(sigma)
    if expected_levels is None:
        expected_levels = sortwt_levels_np(S, sigma) if n > 64 else sortwt_levels_py(list(map(int, S)), sigma)
    bits = np.asarray(t["bits"]).reshape(L, -1) if L else np.zeros((0, 0), dtype=np.uint64)
    for l in range(L):
        if not np.array_equal(bits[l], pack(expected_levels[l], n)):
            fails.append(f"sortwt_level{l}")
            break
    S64 = S.astype(np.uint64)
    for l in range(L):
        k = L - 1 - l
        want = int(np.count_nonzero((S64 >> np.uint64(k)) & np.uint64(1)))
        if int(unpack(bits[l], n).sum()) != want:
            fails.append(f"popcount_level{l}")
            break
    if not np.array_equal(np.asarray(t["C"], dtype=np.uint64), expected_C(S, sigma)):
        fails.append("histogram_C")
    else:
        C = np.asarray(t["C"], dtype=np.int64)
        for l in range(L):
            k = L - 1 - l
            row = unpack(bits[l], n)
            cz = np.concatenate([[0], np.cumsum(row == 0)])
            p = np.arange(1 << l, dtype=np.int64)
            a = C[np.minimum(p << (k + 1), sigma)]
            e = C[np.minimum((p + 1) << (k + 1), sigma)]
            right = C[np.minimum((2 * p + 1) << k, sigma)]
            if not np.array_equal(right - a, cz[e] - cz[a]):
                fails.append(f"node_offsets_level{l}")
                break
    if "rank" in t:
        want = naive_dirs([unpack(bits[l], n) for l in range(L)], n)
        for key in ("rank", "sel1", "sel0", "sel_counts"):
            got = np.asarray(t[key], dtype=np.uint64).reshape(want[key].shape)
            if not np.array_equal(got, want[key]):
                fails.append(f"dirs_{key}")
    return fails


def naive_rank(S: np.ndarray, c: int, i: int) -> int:
    return int(np.count_nonzero(S[: min(i, S.shape[0])] == c))


def naive_select(S: np.ndarray, c: int, k: int) -> int:
    if k <= 0:
        return -1
    pos = np.flatnonzero(S == c)
    return int(pos[k - 1]) if k <= pos.size else -1


def matrix_key(s: int, l: int, L: int) -> int:
    """The top l bits of s read in reverse: bit L-1 weighs 1, bit L-l weighs 2^(l-1)."""
    return sum(((s >> (L - 1 - j)) & 1) << j for j in range(l))


def matrix_levels_py(S, sigma: int):
    """Wavelet matrix levels by pure-Python stable ``sorted`` (tiny inputs)."""
    L = levels(sigma)
    out = []
    for l in range(L):
        T = sorted(S, key=lambda s: matrix_key(s, l, L))
        out.append([(s >> (L - 1 - l)) & 1 for s in T])
    return out


def matrix_levels_np(S: np.ndarray, sigma: int) -> list[np.ndarray]:
    """The same with numpy: the key is built bit by bit, then stably argsorted."""
    L = levels(sigma)
    S64 = S.astype(np.uint64)
    out = []
    for l in range(L):
        key = np.zeros(S.shape[0], dtype=np.uint64)
        for j in range(l):
            key |= ((S64 >> np.uint64(L - 1 - j)) & np.uint64(1)) << np.uint64(j)
        order = np.argsort(key, kind="stable")
        out.append(((S64[order] >> np.uint64(L - 1 - l)) & np.uint64(1)).astype(np.uint8))
    return out


def check_matrix(t: dict, S: np.ndarray, sigma: int, expected_levels=None) -> list[str]:
    """Names of the pins that the wavelet matrix ``t`` ({'bits','zeros',...}) fails."""
    fails = []
    n = S.shape[0]
    L = levels(sigma)
    if expected_levels is None:
        expected_levels = matrix_levels_np(S, sigma) if n > 64 else matrix_levels_py(list(map(int, S)), sigma)
    bits = np.asarray(t["bits"]).reshape(L, -1) if L else np.zeros((0, 0), dtype=np.uint64)
    for l in range(L):
        if not np.array_equal(bits[l], pack(expected_levels[l], n)):
            fails.append(f"matrix_level{l}")
            break
    S64 = S.astype(np.uint64)
    zeros = np.asarray(t["zeros"], dtype=np.uint64).reshape(-1)[:L]
    for l in range(L):
        want = int(np.count_nonzero(((S64 >> np.uint64(L - 1 - l)) & np.uint64(1)) == 0))
        if int(zeros[l]) != want:
            fails.append(f"matrix_zeros{l}")
            break
    if "rank" in t:
        want = naive_dirs([unpack(bits[l], n) for l in range(L)], n)
        for key in ("rank", "sel1", "sel0", "sel_counts"):
            got = np.asarray(t[key], dtype=np.uint64).reshape(want[key].shape)
            if not np.array_equal(got, want[key]):
                fails.append(f"matrix_dirs_{key}")
    return fails


def levels4(sigma: int) -> int:
    return (levels(sigma) + 1) // 2


def digit(s: int, j: int, Lq: int) -> int:
    return (s >> (2 * (Lq - 1 - j))) & 3


def multiary_levels_py(S, sigma: int):
    """4-ary levels by pure-Python stable ``sorted`` (tiny inputs)."""
    Lq = levels4(sigma)
    out = []
    for j in range(Lq):
        T = sorted(S, key=lambda s: s >> (2 * (Lq - j)))
        out.append([digit(s, j, Lq) for s in T])
    return out


def multiary_levels_np(S: np.ndarray, sigma: int) -> list[np.ndarray]:
    Lq = levels4(sigma)
    S64 = S.astype(np.uint64)
    out = []
    for j in range(Lq):
        order = np.argsort(S64 >> np.uint64(2 * (Lq - j)), kind="stable")
        out.append(((S64[order] >> np.uint64(2 * (Lq - 1 - j))) & np.uint64(3)).astype(np.uint8))
    return out


def pack4(entries, n: int) -> np.ndarray:
    """2-bit entries, 32 per 64-bit word, LSB-first."""
    W4 = (n + 31) // 32
    e = np.zeros(W4 * 32, dtype=np.uint64)
    e[:n] = np.asarray(entries, dtype=np.uint64)[:n]
    if W4 == 0:
        return np.zeros(0, dtype=np.uint64)
    shifts = (np.arange(32, dtype=np.uint64) * np.uint64(2))
    return np.bitwise_or.reduce(e.reshape(W4, 32) << shifts, axis=1)


def naive_dirs4(rows: list, n: int) -> dict:
    Lq = len(rows)
    R = (n + RANK_BLOCK_BITS - 1) // RANK_BLOCK_BITS + 1
    cap = (n + SEL_SAMPLE - 1) // SEL_SAMPLE + 1
    rank4 = np.zeros((Lq, R, 4), dtype=np.uint64)
    sel4 = np.full((Lq, 4, cap), n, dtype=np.uint64)
    counts4 = np.zeros((Lq, 4), dtype=np.uint64)
    pos = np.minimum(np.arange(R, dtype=np.int64) * RANK_BLOCK_BITS, n)
    for j, row in enumerate(rows):
        row = np.asarray(row, dtype=np.int64)
        for v in range(4):
            hit = (row == v).astype(np.int64)
            cs = np.concatenate([[0], np.cumsum(hit)])
            rank4[j, :, v] = cs[pos]
            where = np.flatnonzero(hit)[::SEL_SAMPLE]
            sel4[j, v, : where.size] = where
            counts4[j, v] = where.size
    return {"rank4": rank4, "sel4": sel4, "counts4": counts4}


def check_multiary(t: dict, S: np.ndarray, sigma: int) -> list[str]:
    """Names of the pins that the 4-ary tree ``t`` ({'digits','C',...}) fails."""
    fails = []
    n = S.shape[0]
    Lq = levels4(sigma)
    rows = multiary_levels_np(S, sigma) if n > 64 else multiary_levels_py(list(map(int, S)), sigma)
    D = np.asarray(t["digits"], dtype=np.uint64).reshape(Lq, -1) if Lq else np.zeros((0, 0), dtype=np.uint64)
    for j in range(Lq):
        if not np.array_equal(D[j], pack4(rows[j], n)):
            fails.append(f"multiary_level{j}")
            break
    if not np.array_equal(np.asarray(t["C"], dtype=np.uint64), expected_C(S, sigma)):
        fails.append("multiary_C")
    if "rank4" in t:
        want = naive_dirs4(rows, n)
        for key in ("rank4", "sel4", "counts4"):
            if not np.array_equal(np.asarray(t[key], dtype=np.uint64).reshape(want[key].shape), want[key]):
                fails.append(f"multiary_dirs_{key}")
    return fails
