"""ctypes front end of the plain C oracle (wt_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use this module; the GPU library never does.  It shares no
code with the library: it loads its own shared object built from
``wt_oracle.c`` with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wt_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

RANK_BLOCK_BITS = 512
SEL_SAMPLE = 4096

_u64p = ctypes.POINTER(ctypes.c_uint64)


def compile_oracle(out_path: str = LIB, mutant: int | None = None) -> str:
    """Compile wt_oracle.c with gcc into ``out_path`` (optionally a planted mutant)."""
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", out_path, SRC]
    if mutant is not None:
        cmd.insert(1, f"-DORACLE_MUTANT={int(mutant)}")
    subprocess.run(cmd, check=True)
    return out_path


def _declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    lib.oracle_levels.restype = ctypes.c_uint32
    lib.oracle_levels.argtypes = [ctypes.c_uint64]
    lib.oracle_build.restype = ctypes.c_int
    lib.oracle_build.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                 _u64p, _u64p]
    lib.oracle_rank_select.restype = ctypes.c_int
    lib.oracle_rank_select.argtypes = [_u64p, ctypes.c_uint64, ctypes.c_uint32, _u64p, _u64p, _u64p, _u64p]
    lib.oracle_access_naive.restype = ctypes.c_uint64
    lib.oracle_access_naive.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64]
    lib.oracle_rank_naive.restype = ctypes.c_uint64
    lib.oracle_rank_naive.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_uint64]
    lib.oracle_select_naive.restype = ctypes.c_int64
    lib.oracle_select_naive.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_uint64]
    for name in ("oracle_access_tree",):
        getattr(lib, name).restype = ctypes.c_uint64
        getattr(lib, name).argtypes = [_u64p, _u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    lib.oracle_rank_tree.restype = ctypes.c_uint64
    lib.oracle_rank_tree.argtypes = [_u64p, _u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_uint64]
    lib.oracle_select_tree.restype = ctypes.c_int64
    lib.oracle_select_tree.argtypes = [_u64p, _u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_uint64]
    lib.oracle_build_matrix.restype = ctypes.c_int
    lib.oracle_build_matrix.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                        _u64p, _u64p]
    lib.oracle_access_matrix.restype = ctypes.c_uint64
    lib.oracle_access_matrix.argtypes = [_u64p, _u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    lib.oracle_rank_matrix.restype = ctypes.c_uint64
    lib.oracle_rank_matrix.argtypes = [_u64p, _u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_uint64]
    lib.oracle_select_matrix.restype = ctypes.c_int64
    lib.oracle_select_matrix.argtypes = [_u64p, _u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_uint64]
    lib.oracle_levels4.restype = ctypes.c_uint32
    lib.oracle_levels4.argtypes = [ctypes.c_uint64]
    lib.oracle_build_multiary.restype = ctypes.c_int
    lib.oracle_build_multiary.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                          _u64p, _u64p]
    lib.oracle_rank_select4.restype = ctypes.c_int
    lib.oracle_rank_select4.argtypes = [_u64p, ctypes.c_uint64, ctypes.c_uint32, _u64p, _u64p, _u64p]
    lib.oracle_access_multiary.restype = ctypes.c_uint64
    lib.oracle_access_multiary.argtypes = [_u64p, _u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    lib.oracle_rank_multiary.restype = ctypes.c_uint64
    lib.oracle_rank_multiary.argtypes = [_u64p, _u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_uint64]
    lib.oracle_select_multiary.restype = ctypes.c_int64
    lib.oracle_select_multiary.argtypes = [_u64p, _u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.c_uint64]
    return lib


_LIBS: dict[str, ctypes.CDLL] = {}


def _declare_huffman(lib: ctypes.CDLL) -> None:
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.oracle_huffman_lengths.restype = ctypes.c_uint32
    lib.oracle_huffman_lengths.argtypes = [_u64p, ctypes.c_uint32, u32p]
    lib.oracle_huffman_codes.restype = None
    lib.oracle_huffman_codes.argtypes = [u32p, ctypes.c_uint32, _u64p]
    lib.oracle_build_huffman.restype = ctypes.c_int
    lib.oracle_build_huffman.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, u32p, _u64p,
                                         ctypes.c_uint32, _u64p, _u64p]


def load(path: str = LIB) -> ctypes.CDLL:
    """Load (compiling first if needed) the oracle shared object at ``path``."""
    if path not in _LIBS:
        if path == LIB and (not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            compile_oracle(LIB)
        lib = _declare(ctypes.CDLL(path))
        _declare_huffman(lib)
        _LIBS[path] = lib
    return _LIBS[path]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_u64p)


def levels(sigma: int) -> int:
    return int(load().oracle_levels(sigma))


def sym_bytes_of(S: np.ndarray) -> int:
    return {np.dtype(np.uint8): 1, np.dtype(np.uint16): 2, np.dtype(np.uint32): 4}[S.dtype]


class OracleError(RuntimeError):
    pass


def build(S: np.ndarray, sigma: int, lib_path: str = LIB) -> dict:
    """Build bits and C.  Returns {'L', 'W', 'bits' (L, W) uint64, 'C' (sigma+1,) uint64}."""
    lib = load(lib_path)
    S = np.ascontiguousarray(S)
    n = int(S.shape[0])
    L = int(lib.oracle_levels(sigma))
    W = (n + 63) // 64
    bits = np.zeros(max(L * W, 1), dtype=np.uint64)
    C = np.zeros(sigma + 1, dtype=np.uint64)
    rc = lib.oracle_build(S.ctypes.data_as(ctypes.c_void_p), n, sigma, sym_bytes_of(S), _ptr(bits), _ptr(C))
    if rc != 0:
        raise OracleError(f"oracle_build returned {rc}")
    return {"L": L, "W": W, "n": n, "sigma": sigma, "bits": bits[: L * W].reshape(L, W), "C": C}


def rank_select(bits: np.ndarray, n: int, L: int, lib_path: str = LIB) -> dict:
    """Directories over (L, W) level bits (see oracle_rank_select for the format)."""
    lib = load(lib_path)
    W = (n + 63) // 64
    flat = np.ascontiguousarray(bits, dtype=np.uint64).reshape(-1)
    if flat.size == 0:
        flat = np.zeros(1, dtype=np.uint64)
    rank_len = (n + RANK_BLOCK_BITS - 1) // RANK_BLOCK_BITS + 1
    cap = (n + SEL_SAMPLE - 1) // SEL_SAMPLE + 1
    rank = np.zeros(max(L * rank_len, 1), dtype=np.uint64)
    sel1 = np.zeros(max(L * cap, 1), dtype=np.uint64)
    sel0 = np.zeros(max(L * cap, 1), dtype=np.uint64)
    counts = np.zeros(max(2 * L, 1), dtype=np.uint64)
    lib.oracle_rank_select(_ptr(flat), n, L, _ptr(rank), _ptr(sel1), _ptr(sel0), _ptr(counts))
    return {
        "rank": rank[: L * rank_len].reshape(L, rank_len),
        "sel1": sel1[: L * cap].reshape(L, cap),
        "sel0": sel0[: L * cap].reshape(L, cap),
        "sel_counts": counts[: 2 * L],
    }


def build_all(S: np.ndarray, sigma: int, lib_path: str = LIB) -> dict:
    t = build(S, sigma, lib_path)
    t.update(rank_select(t["bits"], t["n"], t["L"], lib_path))
    return t


# ---- queries ---------------------------------------------------------------

def access_naive(S: np.ndarray, i: int) -> int:
    return int(load().oracle_access_naive(S.ctypes.data_as(ctypes.c_void_p), sym_bytes_of(S), i))


def rank_naive(S: np.ndarray, c: int, i: int) -> int:
    return int(load().oracle_rank_naive(S.ctypes.data_as(ctypes.c_void_p), sym_bytes_of(S), S.shape[0], c, i))


def select_naive(S: np.ndarray, c: int, k: int) -> int:
    return int(load().oracle_select_naive(S.ctypes.data_as(ctypes.c_void_p), sym_bytes_of(S), S.shape[0], c, k))


def _tree_args(t: dict):
    bits = np.ascontiguousarray(t["bits"], dtype=np.uint64).reshape(-1)
    if bits.size == 0:
        bits = np.zeros(1, dtype=np.uint64)
    return bits, np.ascontiguousarray(t["C"], dtype=np.uint64)


def access_tree(t: dict, i: int, lib_path: str = LIB) -> int:
    bits, C = _tree_args(t)
    return int(load(lib_path).oracle_access_tree(_ptr(bits), _ptr(C), t["n"], t["sigma"], i))


def rank_tree(t: dict, c: int, i: int, lib_path: str = LIB) -> int:
    bits, C = _tree_args(t)
    return int(load(lib_path).oracle_rank_tree(_ptr(bits), _ptr(C), t["n"], t["sigma"], c, i))


def select_tree(t: dict, c: int, k: int, lib_path: str = LIB) -> int:
    bits, C = _tree_args(t)
    return int(load(lib_path).oracle_select_tree(_ptr(bits), _ptr(C), t["n"], t["sigma"], c, k))


# ---- wavelet matrix ----------------------------------------------------------

def build_matrix(S: np.ndarray, sigma: int, lib_path: str = LIB) -> dict:
    """Wavelet matrix bits and per-level zero counts:
    {'L', 'W', 'n', 'sigma', 'bits' (L, W) uint64, 'zeros' (L,) uint64}."""
    lib = load(lib_path)
    S = np.ascontiguousarray(S)
    n = int(S.shape[0])
    L = int(lib.oracle_levels(sigma))
    W = (n + 63) // 64
    bits = np.zeros(max(L * W, 1), dtype=np.uint64)
    zeros = np.zeros(max(L, 1), dtype=np.uint64)
    rc = lib.oracle_build_matrix(S.ctypes.data_as(ctypes.c_void_p), n, sigma, sym_bytes_of(S), _ptr(bits),
                                 _ptr(zeros))
    if rc != 0:
        raise OracleError(f"oracle_build_matrix returned {rc}")
    return {"L": L, "W": W, "n": n, "sigma": sigma, "bits": bits[: L * W].reshape(L, W), "zeros": zeros[:L]}


def build_matrix_all(S: np.ndarray, sigma: int, lib_path: str = LIB) -> dict:
    """Wavelet matrix with the directories of its level bitmaps."""
    t = build_matrix(S, sigma, lib_path)
    t.update(rank_select(t["bits"], t["n"], t["L"], lib_path))
    return t


def _matrix_args(t: dict):
    bits = np.ascontiguousarray(t["bits"], dtype=np.uint64).reshape(-1)
    if bits.size == 0:
        bits = np.zeros(1, dtype=np.uint64)
    zeros = np.ascontiguousarray(t["zeros"], dtype=np.uint64)
    if zeros.size == 0:
        zeros = np.zeros(1, dtype=np.uint64)
    return bits, zeros


def access_matrix(t: dict, i: int, lib_path: str = LIB) -> int:
    bits, zeros = _matrix_args(t)
    return int(load(lib_path).oracle_access_matrix(_ptr(bits), _ptr(zeros), t["n"], t["sigma"], i))


def rank_matrix(t: dict, c: int, i: int, lib_path: str = LIB) -> int:
    bits, zeros = _matrix_args(t)
    return int(load(lib_path).oracle_rank_matrix(_ptr(bits), _ptr(zeros), t["n"], t["sigma"], c, i))


def select_matrix(t: dict, c: int, k: int, lib_path: str = LIB) -> int:
    bits, zeros = _matrix_args(t)
    return int(load(lib_path).oracle_select_matrix(_ptr(bits), _ptr(zeros), t["n"], t["sigma"], c, k))


# ---- multiary wavelet tree (d = 4) -----------------------------------------

def build_multiary(S: np.ndarray, sigma: int, lib_path: str = LIB) -> dict:
    """4-ary tree: {'Lq', 'W4', 'n', 'sigma', 'digits' (Lq, W4) uint64, 'C'}."""
    lib = load(lib_path)
    S = np.ascontiguousarray(S)
    n = int(S.shape[0])
    Lq = int(lib.oracle_levels4(sigma))
    W4 = (n + 31) // 32
    digits = np.zeros(max(Lq * W4, 1), dtype=np.uint64)
    C = np.zeros(sigma + 1, dtype=np.uint64)
    rc = lib.oracle_build_multiary(S.ctypes.data_as(ctypes.c_void_p), n, sigma, sym_bytes_of(S), _ptr(digits),
                                   _ptr(C))
    if rc != 0:
        raise OracleError(f"oracle_build_multiary returned {rc}")
    return {"Lq": Lq, "W4": W4, "n": n, "sigma": sigma, "digits": digits[: Lq * W4].reshape(Lq, W4), "C": C}


def rank_select4(digits: np.ndarray, n: int, Lq: int, lib_path: str = LIB) -> dict:
    """Directories of 4-ary levels (see oracle_rank_select4 for the format)."""
    lib = load(lib_path)
    flat = np.ascontiguousarray(digits, dtype=np.uint64).reshape(-1)
    if flat.size == 0:
        flat = np.zeros(1, dtype=np.uint64)
    R = (n + RANK_BLOCK_BITS - 1) // RANK_BLOCK_BITS + 1
    cap = (n + SEL_SAMPLE - 1) // SEL_SAMPLE + 1
    rank4 = np.zeros(max(Lq * R * 4, 1), dtype=np.uint64)
    sel4 = np.zeros(max(Lq * 4 * cap, 1), dtype=np.uint64)
    counts4 = np.zeros(max(Lq * 4, 1), dtype=np.uint64)
    lib.oracle_rank_select4(_ptr(flat), n, Lq, _ptr(rank4), _ptr(sel4), _ptr(counts4))
    return {"rank4": rank4[: Lq * R * 4].reshape(Lq, R, 4), "sel4": sel4[: Lq * 4 * cap].reshape(Lq, 4, cap),
            "counts4": counts4[: Lq * 4].reshape(Lq, 4)}


def build_multiary_all(S: np.ndarray, sigma: int, lib_path: str = LIB) -> dict:
    t = build_multiary(S, sigma, lib_path)
    t.update(rank_select4(t["digits"], t["n"], t["Lq"], lib_path))
    return t


def _multiary_args(t: dict):
    d = np.ascontiguousarray(t["digits"], dtype=np.uint64).reshape(-1)
    if d.size == 0:
        d = np.zeros(1, dtype=np.uint64)
    return d, np.ascontiguousarray(t["C"], dtype=np.uint64)


def access_multiary(t: dict, i: int, lib_path: str = LIB) -> int:
    d, C = _multiary_args(t)
    return int(load(lib_path).oracle_access_multiary(_ptr(d), _ptr(C), t["n"], t["sigma"], i))


def rank_multiary(t: dict, c: int, i: int, lib_path: str = LIB) -> int:
    d, C = _multiary_args(t)
    return int(load(lib_path).oracle_rank_multiary(_ptr(d), _ptr(C), t["n"], t["sigma"], c, i))


def select_multiary(t: dict, c: int, k: int, lib_path: str = LIB) -> int:
    d, C = _multiary_args(t)
    return int(load(lib_path).oracle_select_multiary(_ptr(d), _ptr(C), t["n"], t["sigma"], c, k))


# ---- Huffman-shaped tree (section "Extensions"; readings in wt_oracle.c) ---
HUFF_MAX_SIGMA = 256


def huffman_lengths(w: np.ndarray, lib_path: str = LIB) -> tuple[np.ndarray, int]:
    """Code lengths (uint32 per symbol, 0 when absent) and the height."""
    w = np.ascontiguousarray(w, dtype=np.uint64)
    sigma = int(w.size)
    if not 1 <= sigma <= HUFF_MAX_SIGMA:
        raise OracleError("the Huffman-shaped tree takes 1 <= sigma <= 256")
    lens = np.zeros(sigma, dtype=np.uint32)
    h = load(lib_path).oracle_huffman_lengths(_ptr(w), sigma, lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return lens, int(h)


def huffman_codes(lens: np.ndarray, lib_path: str = LIB) -> np.ndarray:
    """Canonical codes, left-aligned in 64 bits (uint64 per symbol, 0 when absent)."""
    lens = np.ascontiguousarray(lens, dtype=np.uint32)
    codes = np.zeros(lens.size, dtype=np.uint64)
    load(lib_path).oracle_huffman_codes(lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), lens.size,
                                        _ptr(codes))
    return codes


def build_huffman(S: np.ndarray, sigma: int, lib_path: str = LIB) -> dict:
    """Huffman-shaped tree of byte sequence S: {'lens', 'codes', 'h', 'W', 'n', 'nd' (h,), 'bits' (h, W)}."""
    S = np.ascontiguousarray(S)
    if S.dtype != np.uint8:
        raise OracleError("the Huffman-shaped tree takes byte symbols")
    n = int(S.size)
    if n and int(S.max()) >= sigma:
        raise OracleError("symbol out of range")
    w = np.bincount(S, minlength=sigma).astype(np.uint64)[:sigma]
    lens, h = huffman_lengths(w, lib_path)
    codes = huffman_codes(lens, lib_path)
    W = (n + 63) // 64
    bits = np.zeros(max(h * W, 1), dtype=np.uint64)
    nd = np.zeros(max(h, 1), dtype=np.uint64)
    rc = load(lib_path).oracle_build_huffman(S.ctypes.data_as(ctypes.c_void_p), n, sigma,
                                             lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), _ptr(codes),
                                             h, _ptr(bits), _ptr(nd))
    if rc != 0:
        raise OracleError(f"oracle_build_huffman returned {rc}")
    return {"sigma": sigma, "n": n, "W": W, "h": h, "lens": lens, "codes": codes, "weights": w,
            "nd": nd[:h], "bits": bits[: h * W].reshape(h, W)}


def build_huffman_all(S: np.ndarray, sigma: int, lib_path: str = LIB) -> dict:
    """build_huffman plus directories over each level's nd[d] bits, at the
    per-level strides of an n-symbol tree: rank rows of ceil(n/512)+1
    entries (entries past the level's end repeat its total), select rows of
    ceil(n/4096)+1 entries (unused ones hold nd[d]), sel_counts[d] for the
    ones and sel_counts[h + d] for the zeros of level d."""
    t = build_huffman(S, sigma, lib_path)
    n, h = t["n"], t["h"]
    rank_len = (n + RANK_BLOCK_BITS - 1) // RANK_BLOCK_BITS + 1
    cap = (n + SEL_SAMPLE - 1) // SEL_SAMPLE + 1
    rank = np.zeros((h, rank_len), dtype=np.uint64)
    sel1 = np.zeros((h, cap), dtype=np.uint64)
    sel0 = np.zeros((h, cap), dtype=np.uint64)
    counts = np.zeros(2 * h, dtype=np.uint64)
    for d in range(h):
        m = int(t["nd"][d])
        r = rank_select(t["bits"][d, : (m + 63) // 64], m, 1, lib_path)
        rl = r["rank"].shape[1]
        rank[d, :rl] = r["rank"][0]
        rank[d, rl:] = r["rank"][0, -1]
        cl = r["sel1"].shape[1]
        sel1[d, :cl], sel1[d, cl:] = r["sel1"][0], m
        sel0[d, :cl], sel0[d, cl:] = r["sel0"][0], m
        counts[d], counts[h + d] = r["sel_counts"][0], r["sel_counts"][1]
    t.update({"rank": rank, "sel1": sel1, "sel0": sel0, "sel_counts": counts})
    return t
