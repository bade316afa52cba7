"""CPU tests of the C-ABI library: it loads, exports what include/wt.h declares,
plans sizes correctly and rejects bad arguments synchronously (no GPU work)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1407_8142_amd import wt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|uint64_t)\s+(wt_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("wt_plan", "wt_build", "wt_build_rank_select", "wt_access", "wt_rank", "wt_select",
                     "wt_status_get"):
        assert required in names
    assert sorted(wt.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = wt.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", wt.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(wt_\w+)$", out, flags=re.M))
    for name in declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_header_compiles_as_c():
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c", HEADER], check=True)


@pytest.mark.parametrize("n,sigma,b,L", [(0, 1, 1, 0), (1, 2, 1, 1), (100, 3, 1, 2), (1 << 20, 256, 1, 8),
                                         (1 << 28, 256, 1, 8), (10, 257, 2, 9), (1 << 27, 1 << 16, 4, 16),
                                         (1 << 27, 1 << 20, 4, 20), (5, (1 << 20) + 1, 4, 21),
                                         (5, 1 << 16, 2, 16)])
def test_plan_sizes(n, sigma, b, L):
    lay = wt.plan(n, sigma, b)
    assert lay.L == L
    W = (n + 63) // 64
    assert lay.words_per_level == W and lay.bits_words == L * W
    assert lay.C_len == sigma + 1
    assert lay.rank_len == (n + 511) // 512 + 1
    assert lay.sel_cap == (n + 4095) // 4096 + 1
    assert lay.sel_counts_len == 2 * L
    assert lay.scratch_bytes % 256 == 0 and lay.scratch_bytes >= 256
    # two ping-pong copies of the sequence at the narrowed width when L >= 3
    mid = 1 if L <= 8 else (2 if L <= 16 else 4)
    if L >= 3:
        assert lay.scratch_bytes >= 2 * n * mid
    assert lay.rs_scratch_bytes == wt.lib().wt_rank_select_scratch_bytes(n, L)


@pytest.mark.parametrize("n,sigma,b", [(10, 0, 1), (10, 257, 1), (10, 65537, 2), (10, 5, 3), (1 << 40, 4, 1),
                                       (10, (1 << 31) + 1, 4)])
def test_plan_rejects(n, sigma, b):
    with pytest.raises(wt.WTError) as e:
        wt.plan(n, sigma, b)
    assert e.value.rc in (wt.WT_ERR_ARG, wt.WT_ERR_RANGE)


def test_build_argument_errors_are_synchronous():
    lib = wt.lib()
    out = wt.Outputs()
    # null outputs
    assert lib.wt_build(ctypes.c_void_p(16), 10, 4, 1, None, ctypes.c_void_p(256), 1 << 20, None) == wt.WT_ERR_ARG
    # C missing
    assert lib.wt_build(ctypes.c_void_p(16), 10, 4, 1, ctypes.byref(out), ctypes.c_void_p(256), 1 << 20,
                        None) == wt.WT_ERR_ARG
    out.C = ctypes.c_void_p(4096)
    out.bits = ctypes.c_void_p(8192)
    # misaligned input
    assert lib.wt_build(ctypes.c_void_p(17), 10, 4, 1, ctypes.byref(out), ctypes.c_void_p(256), 1 << 20,
                        None) == wt.WT_ERR_ARG
    # directories half given
    out.rank = ctypes.c_void_p(12288)
    assert lib.wt_build(ctypes.c_void_p(16), 10, 4, 1, ctypes.byref(out), ctypes.c_void_p(256), 1 << 20,
                        None) == wt.WT_ERR_ARG
    out.rank = None
    # scratch too small
    assert lib.wt_build(ctypes.c_void_p(16), 1000, 256, 1, ctypes.byref(out), ctypes.c_void_p(256), 64,
                        None) == wt.WT_ERR_SCRATCH
    # width / sigma mismatch
    assert lib.wt_build(ctypes.c_void_p(16), 10, 300, 1, ctypes.byref(out), ctypes.c_void_p(256), 1 << 20,
                        None) == wt.WT_ERR_ARG
    # rank/select: missing outputs, small scratch
    assert lib.wt_build_rank_select(ctypes.c_void_p(16), 100, 3, None, None, None, None, ctypes.c_void_p(256),
                                    1 << 20, None) == wt.WT_ERR_ARG
    p = ctypes.c_void_p(4096)
    assert lib.wt_build_rank_select(ctypes.c_void_p(16), 100000, 3, p, p, p, p, ctypes.c_void_p(256), 8,
                                    None) == wt.WT_ERR_SCRATCH
    # queries: null view / null buffers
    assert lib.wt_access(None, None, 5, None, None) == wt.WT_ERR_ARG
    v = wt.View()
    v.C = ctypes.c_void_p(4096)
    v.n, v.sigma, v.L = 10, 4, 2
    assert lib.wt_rank(ctypes.byref(v), None, None, 5, None, None) == wt.WT_ERR_ARG
    # empty batches are no-ops
    v.bits = v.rank = v.sel1 = v.sel0 = ctypes.c_void_p(4096)
    assert lib.wt_select(ctypes.byref(v), None, None, 0, None, None) == wt.WT_OK
