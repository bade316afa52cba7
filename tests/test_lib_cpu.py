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
                                         (5, 1 << 16, 2, 16), (10, (1 << 31) + 1, 4, 32), (1000, 1 << 32, 4, 32),
                                         (1 << 20, 1 << 31, 4, 31)])
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
                                       (10, (1 << 32) + 1, 4)])
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


def test_noalloc_refuses_plans_beyond_its_array():
    """wt_build_noalloc refuses a plan larger than its static array (and bad
    arguments) synchronously, before touching the device."""
    lib = wt.lib()
    out = wt.Outputs()
    out.C = ctypes.c_void_p(4096)
    out.bits = ctypes.c_void_p(8192)
    n = 80 << 20
    assert wt.plan(n, 256, 1).scratch_bytes > wt.NOALLOC_SCRATCH_BYTES
    assert lib.wt_build_noalloc(ctypes.c_void_p(16), n, 256, 1, ctypes.byref(out), None, None) == wt.WT_ERR_SCRATCH
    assert lib.wt_build_noalloc(ctypes.c_void_p(16), 10, 300, 1, ctypes.byref(out), None, None) == wt.WT_ERR_ARG
    assert lib.wt_build_noalloc(ctypes.c_void_p(16), 10, 0, 1, ctypes.byref(out), None, None) == wt.WT_ERR_ARG


def _job(n, sigma, b):
    return wt.Job(None, n, sigma, b, 0, wt.Outputs())


def test_batch_plan_queue_shape():
    """The queue holds, in phases: level-0 histogram tiles of the jobs
    counted tile by tile, one whole-job histogram item per job whose
    alphabet needs packed LDS bins (5120 <= sigma <= 2^16), one table item
    per job, then per level the byte-symbol tiles and the wider tiles of
    every job that has that level (16 KiB tiles), then one fused-segment item
    per (8 KiB - 32 positions) at the job's narrowed width (the segment stride)."""
    spec = [(0, 4, 1), (1, 1, 1), (100000, 256, 1), (20000, 1 << 16, 2), (5000, 1 << 20, 4), (70000, 5, 1),
            (30000, 6000, 2), (9000, 200, 4)]
    lay = wt.batch_plan([_job(*s) for s in spec])
    tiles = lambda n, w: -(-n // (16384 // w))
    L = lambda s: 0 if s == 1 else (s - 1).bit_length()
    mid = lambda l: 1 if l <= 8 else (2 if l <= 16 else 4)
    job_hist = lambda n, s: n > 0 and s + 1 > 5120 and s <= 65536
    hist = sum(tiles(n, b) for n, s, b in spec if not job_hist(n, s))
    jh = sum(1 for n, s, b in spec if job_hist(n, s))
    per_phase = []
    for l in range(max(L(s) for n, s, b in spec if n)):
        for wide in (False, True):
            per_phase.append(sum(tiles(n, b if l == 0 else mid(L(s))) for n, s, b in spec
                                 if n and l < L(s) and ((b if l == 0 else mid(L(s))) > 1) == wide))
    fused = sum(-(-n // (8192 // mid(L(s)) - 32)) for n, s, b in spec if n and L(s) >= 2)
    assert lay.njobs == len(spec)
    assert lay.phases == 3 + len(per_phase) + 1
    assert lay.items == hist + jh + len(spec) + sum(per_phase) + fused
    firsts = [0, hist, hist + jh, hist + jh + len(spec)]
    for c in per_phase:
        firsts.append(firsts[-1] + c)
    firsts.append(firsts[-1] + fused)
    assert list(lay.phase_first)[:lay.phases + 1] == firsts
    assert lay.scratch_bytes % 256 == 0 and lay.clear_bytes <= lay.scratch_bytes
    assert lay.off_jobs >= lay.clear_bytes


@pytest.mark.parametrize("spec,rc", [([(1 << 32, 4, 1)], wt.WT_ERR_RANGE), ([(10, 300, 1)], wt.WT_ERR_ARG),
                                     ([(10, 0, 1)], wt.WT_ERR_ARG), ([(10, 4, 3)], wt.WT_ERR_ARG),
                                     ([(10, 4, 1), (10, 1 << 31, 4)], wt.WT_ERR_RANGE)])
def test_batch_plan_rejects(spec, rc):
    arr = (wt.Job * len(spec))(*[_job(*s) for s in spec])
    lay = wt.BatchLayout()
    assert wt.lib().wt_batch_plan(arr, len(spec), ctypes.byref(lay)) == rc


def test_batch_prepare_rejects_bad_arguments():
    """Rejected before any device work: NULL or misaligned scratch, a short
    scratch, and a job without directory buffers."""
    jobs = [_job(100, 4, 1)]
    lay = wt.batch_plan(jobs)
    arr = (wt.Job * 1)(*jobs)
    prep = wt.lib().wt_batch_prepare
    assert prep(arr, 1, ctypes.byref(lay), None, lay.scratch_bytes, None) == wt.WT_ERR_ARG
    assert prep(arr, 1, ctypes.byref(lay), ctypes.c_void_p(16), lay.scratch_bytes, None) == wt.WT_ERR_ARG
    assert prep(arr, 1, ctypes.byref(lay), ctypes.c_void_p(4096), lay.scratch_bytes - 1, None) == wt.WT_ERR_SCRATCH
    assert prep(arr, 1, ctypes.byref(lay), ctypes.c_void_p(4096), lay.scratch_bytes, None) == wt.WT_ERR_ARG


def test_matrix_argument_errors_are_synchronous():
    """wt_build_matrix and the matrix queries reject bad arguments before any
    device work (no GPU needed)."""
    lib = wt.lib()
    out = wt.Outputs()
    out.C = ctypes.c_void_p(4096)
    out.bits = ctypes.c_void_p(8192)
    # zero counts missing while there are levels
    assert lib.wt_build_matrix(ctypes.c_void_p(16), 10, 4, 1, ctypes.byref(out), None, ctypes.c_void_p(256),
                               1 << 20, None) == wt.WT_ERR_ARG
    # the rest as for wt_build: misaligned input, small scratch
    z = ctypes.c_void_p(12288)
    assert lib.wt_build_matrix(ctypes.c_void_p(17), 10, 4, 1, ctypes.byref(out), z, ctypes.c_void_p(256),
                               1 << 20, None) == wt.WT_ERR_ARG
    assert lib.wt_build_matrix(ctypes.c_void_p(16), 1000, 256, 1, ctypes.byref(out), z, ctypes.c_void_p(256), 64,
                               None) == wt.WT_ERR_SCRATCH
    # queries: null view, missing zero counts, null buffers; empty batches are no-ops
    assert lib.wt_matrix_access(None, None, 5, None, None) == wt.WT_ERR_ARG
    v = wt.MatrixView()
    v.n, v.sigma, v.L = 10, 4, 2
    v.bits = v.rank = v.sel1 = v.sel0 = ctypes.c_void_p(4096)
    assert lib.wt_matrix_rank(ctypes.byref(v), None, None, 5, None, None) == wt.WT_ERR_ARG
    v.zeros = ctypes.c_void_p(4096)
    assert lib.wt_matrix_rank(ctypes.byref(v), None, None, 5, None, None) == wt.WT_ERR_ARG
    assert lib.wt_matrix_select(ctypes.byref(v), None, None, 0, None, None) == wt.WT_OK
    assert lib.wt_matrix_access(ctypes.byref(v), None, 0, None, None) == wt.WT_OK


def test_multiary_argument_errors_are_synchronous():
    lib = wt.lib()
    out = wt.MultiaryOutputs()
    # wider symbols are out of range for the 4-ary build
    assert lib.wt_build_multiary(ctypes.c_void_p(16), 10, 300, 2, ctypes.byref(out), ctypes.c_void_p(256),
                                 1 << 20, None) == wt.WT_ERR_RANGE
    # C missing, then directories missing
    assert lib.wt_build_multiary(ctypes.c_void_p(16), 10, 200, 1, ctypes.byref(out), ctypes.c_void_p(256),
                                 1 << 20, None) == wt.WT_ERR_ARG
    out.C = ctypes.c_void_p(4096)
    assert lib.wt_build_multiary(ctypes.c_void_p(16), 10, 200, 1, ctypes.byref(out), ctypes.c_void_p(256),
                                 1 << 20, None) == wt.WT_ERR_ARG
    out.digits = out.rank4 = out.sel4 = out.counts4 = ctypes.c_void_p(8192)
    assert lib.wt_build_multiary(ctypes.c_void_p(16), 100000, 200, 1, ctypes.byref(out), ctypes.c_void_p(256), 64,
                                 None) == wt.WT_ERR_SCRATCH
    assert lib.wt_multiary_access(None, None, 5, None, None) == wt.WT_ERR_ARG
    v = wt.MultiaryView()
    v.C = ctypes.c_void_p(4096)
    v.n, v.sigma, v.Lq = 10, 16, 2
    assert lib.wt_multiary_rank(ctypes.byref(v), None, None, 5, None, None) == wt.WT_ERR_ARG


def test_huffman_plan_and_argument_errors_are_synchronous():
    lib = wt.lib()
    hb, sb = ctypes.c_uint32(0), ctypes.c_uint64(0)
    # height bound: the largest d with F(d+2) <= n, at most sigma - 1
    for n, sigma, want in [(0, 256, 0), (1, 256, 0), (2, 256, 1), (3, 256, 2), (4, 256, 2), (5, 256, 3),
                           (1 << 28, 256, 40), (1 << 28, 5, 4), (1000, 1, 0)]:
        assert lib.wt_huffman_plan(n, sigma, 0, ctypes.byref(hb), None, None) == wt.WT_OK
        assert hb.value == want, (n, sigma, hb.value)
    tb = ctypes.c_uint64(0)
    assert lib.wt_huffman_plan(1 << 20, 256, 10, None, ctypes.byref(sb), ctypes.byref(tb)) == wt.WT_OK
    assert sb.value > 2 << 20 and tb.value > 0
    assert lib.wt_huffman_plan(1 << 20, 257, 10, None, None, None) == wt.WT_ERR_RANGE
    assert lib.wt_huffman_plan(1 << 32, 256, 10, None, None, None) == wt.WT_ERR_RANGE
    assert lib.wt_huffman_plan(100, 256, 49, None, None, None) == wt.WT_ERR_RANGE
    out = wt.HuffmanOutputs()
    h = ctypes.c_uint32(0)
    assert lib.wt_build_huffman(ctypes.c_void_p(16), 10, 300, ctypes.byref(out), 4, ctypes.byref(h),
                                ctypes.c_void_p(256), 1 << 20, None) == wt.WT_ERR_RANGE
    assert lib.wt_build_huffman(ctypes.c_void_p(16), 10, 200, ctypes.byref(out), 4, ctypes.byref(h),
                                ctypes.c_void_p(256), 1 << 20, None) == wt.WT_ERR_ARG
    out.C = out.lens = out.codes = out.tables = ctypes.c_void_p(4096)
    assert lib.wt_build_huffman(ctypes.c_void_p(16), 10, 200, ctypes.byref(out), 4, ctypes.byref(h),
                                ctypes.c_void_p(256), 1 << 20, None) == wt.WT_ERR_ARG
    out.bits = out.rank = out.sel1 = out.sel0 = out.sel_counts = out.nd = ctypes.c_void_p(8192)
    assert lib.wt_build_huffman(ctypes.c_void_p(17), 10, 200, ctypes.byref(out), 4, ctypes.byref(h),
                                ctypes.c_void_p(256), 1 << 20, None) == wt.WT_ERR_ARG
    assert lib.wt_build_huffman(ctypes.c_void_p(16), 100000, 200, ctypes.byref(out), 4, ctypes.byref(h),
                                ctypes.c_void_p(256), 64, None) == wt.WT_ERR_SCRATCH
    assert lib.wt_huffman_access(None, None, 5, None, None) == wt.WT_ERR_ARG
    v = wt.HuffmanView()
    v.n, v.sigma, v.h = 10, 300, 2
    v.tables = ctypes.c_void_p(4096)
    assert lib.wt_huffman_rank(ctypes.byref(v), None, None, 5, None, None) == wt.WT_ERR_ARG  # sigma > 256
    v.sigma = 200
    assert lib.wt_huffman_select(ctypes.byref(v), None, None, 5, None, None) == wt.WT_ERR_ARG  # no bits


def test_sort_scratch_and_argument_errors_are_synchronous():
    lib = wt.lib()
    assert lib.wt_sort_scratch_bytes(1000, 300) == 0
    assert lib.wt_sort_scratch_bytes(1 << 32, 256) == 0
    # the scratch holds L sorted copies of S
    assert lib.wt_sort_scratch_bytes(1 << 20, 256) >= 8 << 20
    out = wt.Outputs()
    assert lib.wt_build_sort(ctypes.c_void_p(16), 10, 300, 2, ctypes.byref(out), ctypes.c_void_p(256), 1 << 20,
                             None) == wt.WT_ERR_RANGE
    assert lib.wt_build_sort(ctypes.c_void_p(16), 10, 200, 1, ctypes.byref(out), ctypes.c_void_p(256), 1 << 20,
                             None) == wt.WT_ERR_ARG
    out.C = ctypes.c_void_p(4096)
    out.bits = out.rank = out.sel1 = out.sel0 = out.sel_counts = ctypes.c_void_p(8192)
    assert lib.wt_build_sort(ctypes.c_void_p(16), 100000, 200, 1, ctypes.byref(out), ctypes.c_void_p(256), 64,
                             None) == wt.WT_ERR_SCRATCH


@pytest.mark.parametrize("n,sigma,b,path", [
    (0, 256, 1, wt.HIST_NONE),
    (1 << 28, 256, 1, wt.HIST_LEVELS),
    (1 << 20, 146, 1, wt.HIST_LEVELS),
    (1000, 256, 1, wt.HIST_REPLICAS),   # small: fused tail levels, which need C first
    (1 << 20, 300, 2, wt.HIST_REPLICAS),
    (1 << 20, 8192, 2, wt.HIST_REPLICAS),
    (1 << 27, 1 << 16, 4, wt.HIST_SLICES),
    (1 << 27, 1 << 20, 4, wt.HIST_TWO_PHASE),
    ((1 << 25) + 9, (1 << 18) + 1, 4, wt.HIST_TWO_PHASE),
    (1 << 26, 528155, 4, wt.HIST_TWO_PHASE),
    (1000, 1 << 20, 4, wt.HIST_HASH),
])
def test_histogram_path(n, sigma, b, path):
    # the host-side choice of histogram (a 256-CU device is assumed without a GPU)
    assert wt.histogram_path(n, sigma, b) == path



@pytest.mark.parametrize("n,sigma", [(1 << 12, 1 << 20), (1 << 20, 1 << 32), (100_003, (1 << 31) + 1),
                                     (1 << 27, 1 << 30)])
def test_sparse_tables_keep_scratch_small(n, sigma):
    """Alphabets much larger than n (and every L > 30) get node tables over
    the nonempty nodes only: the scratch grows with n, not with 2^L."""
    lay = wt.plan(n, sigma, 4)
    dense_words = 2 << lay.L
    assert lay.scratch_bytes < 8 * dense_words or lay.L > 30
    assert lay.scratch_bytes <= 2 * 4 * n + 64 * n + (64 << 20)


def test_fused_levels_setting():
    """wt_set_fused_levels takes 0 (none), 1 (every level from the first whose
    nodes fit) or m >= 2 (at most the last m levels); a negative value is an
    argument error and leaves the setting alone."""
    lib = wt.lib()
    try:
        for v in (0, 1, 2, 6, 40):
            assert lib.wt_set_fused_levels(v) == wt.WT_OK
        assert lib.wt_set_fused_levels(-1) == wt.WT_ERR_ARG
        with pytest.raises(Exception):
            wt.set_fused_levels(-3)
    finally:
        wt.set_fused_levels(1)
