"""Python binding of libwt.so: argument marshalling only.

Every step of construction and every query runs in the HIP kernels of
libwt.so; torch supplies device memory and the current stream.  Importing
this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwt.so")

WT_OK, WT_ERR_ARG, WT_ERR_SYMBOL, WT_ERR_SCRATCH, WT_ERR_RANGE, WT_ERR_HIP, WT_ERR_NOMEM, WT_ERR_TIMEOUT = \
    0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "WT_OK", -1: "WT_ERR_ARG", -2: "WT_ERR_SYMBOL", -3: "WT_ERR_SCRATCH", -4: "WT_ERR_RANGE",
                -5: "WT_ERR_HIP", -6: "WT_ERR_NOMEM", -7: "WT_ERR_TIMEOUT"}
BATCH_PERSISTENT, BATCH_PER_PHASE = 0, 1
RANK_BLOCK_BITS = 512
SELECT_SAMPLE = 4096

EXPORTS = ["wt_plan", "wt_build", "wt_build_rank_select", "wt_rank_select_scratch_bytes", "wt_status_get",
           "wt_access", "wt_rank", "wt_select", "wt_set_lookback_spin_limit", "wt_timing_enable", "wt_timing_collect",
           "wt_batch_plan", "wt_batch_prepare", "wt_batch_run", "wt_batch_status", "wt_query_multi", "wt_set_fused_levels",
           "wt_set_sliced_histogram", "wt_set_level_pairs", "wt_build_matrix", "wt_matrix_access",
           "wt_matrix_rank", "wt_matrix_select", "wt_build_multiary", "wt_multiary_access", "wt_multiary_rank",
           "wt_multiary_select", "wt_huffman_plan", "wt_build_huffman", "wt_huffman_access", "wt_huffman_rank",
           "wt_huffman_select", "wt_sort_scratch_bytes", "wt_build_sort", "wt_histogram_path", "wt_build_noalloc"]
NOALLOC_SCRATCH_BYTES = 64 << 20  # WT_NOALLOC_SCRATCH_BYTES
Q_ACCESS, Q_RANK, Q_SELECT, Q_BAD = 0, 1, 2, -2
HIST_NONE, HIST_REPLICAS, HIST_HASH, HIST_SLICES, HIST_TWO_PHASE, HIST_LEVELS = 0, 1, 2, 3, 4, 5


class WTError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__(f"{what} failed: {STATUS_NAMES.get(rc, rc)}")
        self.rc = rc


class Layout(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("sigma", ctypes.c_uint64), ("L", ctypes.c_uint32),
                ("sym_bytes", ctypes.c_uint32), ("words_per_level", ctypes.c_uint64),
                ("bits_words", ctypes.c_uint64), ("C_len", ctypes.c_uint64), ("rank_len", ctypes.c_uint64),
                ("sel_cap", ctypes.c_uint64), ("sel_counts_len", ctypes.c_uint64),
                ("scratch_bytes", ctypes.c_uint64), ("rs_scratch_bytes", ctypes.c_uint64)]


class Outputs(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_void_p), ("C", ctypes.c_void_p), ("rank", ctypes.c_void_p),
                ("sel1", ctypes.c_void_p), ("sel0", ctypes.c_void_p), ("sel_counts", ctypes.c_void_p)]


class View(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_void_p), ("C", ctypes.c_void_p), ("rank", ctypes.c_void_p),
                ("sel1", ctypes.c_void_p), ("sel0", ctypes.c_void_p), ("sel_counts", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("sigma", ctypes.c_uint64), ("L", ctypes.c_uint32)]


class MatrixView(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_void_p), ("zeros", ctypes.c_void_p), ("rank", ctypes.c_void_p),
                ("sel1", ctypes.c_void_p), ("sel0", ctypes.c_void_p), ("sel_counts", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("sigma", ctypes.c_uint64), ("L", ctypes.c_uint32)]


class MultiaryOutputs(ctypes.Structure):
    _fields_ = [("digits", ctypes.c_void_p), ("C", ctypes.c_void_p), ("rank4", ctypes.c_void_p),
                ("sel4", ctypes.c_void_p), ("counts4", ctypes.c_void_p)]


class MultiaryView(ctypes.Structure):
    _fields_ = [("digits", ctypes.c_void_p), ("C", ctypes.c_void_p), ("rank4", ctypes.c_void_p),
                ("sel4", ctypes.c_void_p), ("counts4", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("sigma", ctypes.c_uint64), ("Lq", ctypes.c_uint32)]


class HuffmanOutputs(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_void_p), ("C", ctypes.c_void_p), ("rank", ctypes.c_void_p),
                ("sel1", ctypes.c_void_p), ("sel0", ctypes.c_void_p), ("sel_counts", ctypes.c_void_p),
                ("lens", ctypes.c_void_p), ("codes", ctypes.c_void_p), ("nd", ctypes.c_void_p),
                ("tables", ctypes.c_void_p)]


class HuffmanView(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_void_p), ("rank", ctypes.c_void_p), ("sel1", ctypes.c_void_p),
                ("sel0", ctypes.c_void_p), ("tables", ctypes.c_void_p), ("n", ctypes.c_uint64),
                ("sigma", ctypes.c_uint64), ("h", ctypes.c_uint32)]


class Job(ctypes.Structure):
    _fields_ = [("seq", ctypes.c_void_p), ("n", ctypes.c_uint64), ("sigma", ctypes.c_uint64),
                ("sym_bytes", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("out", Outputs)]


class Tune(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32), ("chunk", ctypes.c_uint32),
                ("spin_limit", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class BatchLayout(ctypes.Structure):
    _fields_ = [("scratch_bytes", ctypes.c_uint64), ("clear_bytes", ctypes.c_uint64), ("off_jobs", ctypes.c_uint64),
                ("off_segs", ctypes.c_uint64), ("off_seg_of", ctypes.c_uint64), ("off_list", ctypes.c_uint64),
                ("njobs", ctypes.c_uint32),
                ("nsegs", ctypes.c_uint32), ("items", ctypes.c_uint32), ("phases", ctypes.c_uint32),
                ("phase_first", ctypes.c_uint32 * 72), ("phase_var", ctypes.c_uint32 * 72)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1407_8142_amd/build.py "
                              "(or __graft_entry__.build()) before use")
        L = ctypes.CDLL(LIB_PATH)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        L.wt_plan.argtypes = [u64, u64, i32, ctypes.POINTER(Layout)]
        L.wt_build.argtypes = [vp, u64, u64, i32, ctypes.POINTER(Outputs), vp, u64, vp]
        L.wt_build_noalloc.argtypes = [vp, u64, u64, i32, ctypes.POINTER(Outputs), vp, vp]
        L.wt_build_rank_select.argtypes = [vp, u64, u32, vp, vp, vp, vp, vp, u64, vp]
        L.wt_rank_select_scratch_bytes.argtypes = [u64, u32]
        L.wt_rank_select_scratch_bytes.restype = u64
        L.wt_status_get.argtypes = [vp, vp]
        L.wt_access.argtypes = [ctypes.POINTER(View), vp, u64, vp, vp]
        L.wt_rank.argtypes = [ctypes.POINTER(View), vp, vp, u64, vp, vp]
        L.wt_select.argtypes = [ctypes.POINTER(View), vp, vp, u64, vp, vp]
        L.wt_set_lookback_spin_limit.argtypes = [i32]
        L.wt_timing_enable.argtypes = [i32]
        L.wt_timing_collect.argtypes = [ctypes.POINTER(ctypes.c_float), i32]
        L.wt_batch_plan.argtypes = [ctypes.POINTER(Job), u32, ctypes.POINTER(BatchLayout)]
        L.wt_batch_prepare.argtypes = [ctypes.POINTER(Job), u32, ctypes.POINTER(BatchLayout), vp, u64, vp]
        L.wt_batch_run.argtypes = [ctypes.POINTER(BatchLayout), ctypes.POINTER(Tune), vp, vp]
        L.wt_batch_status.argtypes = [ctypes.POINTER(BatchLayout), vp, ctypes.POINTER(ctypes.c_int32), vp]
        L.wt_query_multi.argtypes = [vp, u32, vp, vp, vp, vp, u64, vp, vp]
        L.wt_histogram_path.argtypes = [u64, u64, i32]
        L.wt_set_fused_levels.argtypes = [i32]
        L.wt_set_sliced_histogram.argtypes = [i32]
        L.wt_set_level_pairs.argtypes = [i32]
        L.wt_build_matrix.argtypes = [vp, u64, u64, i32, ctypes.POINTER(Outputs), vp, vp, u64, vp]
        L.wt_matrix_access.argtypes = [ctypes.POINTER(MatrixView), vp, u64, vp, vp]
        L.wt_matrix_rank.argtypes = [ctypes.POINTER(MatrixView), vp, vp, u64, vp, vp]
        L.wt_matrix_select.argtypes = [ctypes.POINTER(MatrixView), vp, vp, u64, vp, vp]
        L.wt_build_multiary.argtypes = [vp, u64, u64, i32, ctypes.POINTER(MultiaryOutputs), vp, u64, vp]
        L.wt_multiary_access.argtypes = [ctypes.POINTER(MultiaryView), vp, u64, vp, vp]
        L.wt_multiary_rank.argtypes = [ctypes.POINTER(MultiaryView), vp, vp, u64, vp, vp]
        L.wt_multiary_select.argtypes = [ctypes.POINTER(MultiaryView), vp, vp, u64, vp, vp]
        L.wt_huffman_plan.argtypes = [u64, u64, u32, ctypes.POINTER(u32), ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.wt_huffman_access.argtypes = [ctypes.POINTER(HuffmanView), vp, u64, vp, vp]
        L.wt_sort_scratch_bytes.argtypes = [u64, u64]
        L.wt_sort_scratch_bytes.restype = u64
        L.wt_build_sort.argtypes = [vp, u64, u64, i32, ctypes.POINTER(Outputs), vp, u64, vp]
        L.wt_huffman_rank.argtypes = [ctypes.POINTER(HuffmanView), vp, vp, u64, vp, vp]
        L.wt_huffman_select.argtypes = [ctypes.POINTER(HuffmanView), vp, vp, u64, vp, vp]
        L.wt_build_huffman.argtypes = [vp, u64, u64, ctypes.POINTER(HuffmanOutputs), u32, ctypes.POINTER(u32), vp,
                                       u64, vp]
        for f in ("wt_plan", "wt_build", "wt_build_rank_select", "wt_status_get", "wt_access", "wt_rank",
                  "wt_select", "wt_set_lookback_spin_limit", "wt_timing_enable", "wt_timing_collect",
                  "wt_batch_plan", "wt_batch_prepare", "wt_batch_run", "wt_batch_status", "wt_query_multi",
                  "wt_set_fused_levels", "wt_set_sliced_histogram", "wt_set_level_pairs", "wt_build_matrix",
                  "wt_matrix_access", "wt_matrix_rank", "wt_matrix_select", "wt_build_multiary",
                  "wt_multiary_access", "wt_multiary_rank", "wt_multiary_select", "wt_huffman_plan",
                  "wt_build_huffman", "wt_huffman_access", "wt_huffman_rank", "wt_huffman_select",
                  "wt_build_sort", "wt_histogram_path", "wt_build_noalloc"):
            getattr(L, f).restype = i32
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != WT_OK:
        raise WTError(rc, what)


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t: torch.Tensor | None):
    if t is None or t.numel() == 0:
        return None
    return ctypes.c_void_p(t.data_ptr())


def plan(n: int, sigma: int, sym_bytes: int) -> Layout:
    lay = Layout()
    _check(lib().wt_plan(n, sigma, sym_bytes, ctypes.byref(lay)), "wt_plan")
    return lay


@dataclass
class WaveletTree:
    """Device buffers of one built tree (int64 tensors hold the uint64 words)."""
    n: int
    sigma: int
    L: int
    sym_bytes: int
    bits: torch.Tensor
    C: torch.Tensor
    rank: torch.Tensor | None
    sel1: torch.Tensor | None
    sel0: torch.Tensor | None
    sel_counts: torch.Tensor | None
    scratch: torch.Tensor
    layout: Layout

    @staticmethod
    def output_words(n: int, sigma: int, sym_bytes: int) -> tuple[Layout, list[tuple[int, ...]]]:
        """Shapes (in int64 words) of bits, C, rank, sel1, sel0, sel_counts."""
        lay = plan(n, sigma, sym_bytes)
        L, W = lay.L, lay.words_per_level
        return lay, [(L, W), (sigma + 1,), (L, lay.rank_len), (L, lay.sel_cap), (L, lay.sel_cap), (2 * L,)]

    @staticmethod
    def allocate(n: int, sigma: int, sym_bytes: int, directories: bool = True, device="cuda") -> "WaveletTree":
        lay = plan(n, sigma, sym_bytes)
        L, W = lay.L, lay.words_per_level
        e = lambda *shape: torch.empty(*shape, dtype=torch.int64, device=device)
        return WaveletTree(
            n=n, sigma=sigma, L=L, sym_bytes=sym_bytes,
            bits=e(L, W), C=e(sigma + 1),
            rank=e(L, lay.rank_len) if directories else None,
            sel1=e(L, lay.sel_cap) if directories else None,
            sel0=e(L, lay.sel_cap) if directories else None,
            sel_counts=e(2 * L) if directories else None,
            scratch=torch.empty(max(lay.scratch_bytes, 256), dtype=torch.uint8, device=device),
            layout=lay)

    def outputs(self) -> Outputs:
        return Outputs(_ptr(self.bits), _ptr(self.C), _ptr(self.rank), _ptr(self.sel1), _ptr(self.sel0),
                       _ptr(self.sel_counts))

    def view(self) -> View:
        return View(_ptr(self.bits), _ptr(self.C), _ptr(self.rank), _ptr(self.sel1), _ptr(self.sel0),
                    _ptr(self.sel_counts), self.n, self.sigma, self.L)

    # -- construction -------------------------------------------------------
    def build_from(self, seq: torch.Tensor, stream=None) -> "WaveletTree":
        """Launch wt_build on ``seq`` into this tree's buffers (asynchronous)."""
        if not seq.is_cuda:
            raise ValueError("seq must be a device tensor")
        if seq.element_size() != self.sym_bytes or seq.numel() != self.n or not seq.is_contiguous():
            raise ValueError("seq does not match the allocated layout")
        out = self.outputs()
        rc = lib().wt_build(_ptr(seq), self.n, self.sigma, self.sym_bytes, ctypes.byref(out),
                            _ptr(self.scratch), self.scratch.numel(), _stream(stream))
        _check(rc, "wt_build")
        return self

    def build_noalloc_from(self, seq: torch.Tensor, status: torch.Tensor | None = None,
                           stream=None) -> "WaveletTree":
        """Launch wt_build_noalloc on ``seq`` into this tree's outputs (the
        library's static scratch; this tree's scratch is not used).  ``status``
        (a one-element int32 device tensor) receives WT_OK or WT_ERR_SYMBOL."""
        if not seq.is_cuda:
            raise ValueError("seq must be a device tensor")
        if seq.element_size() != self.sym_bytes or seq.numel() != self.n or not seq.is_contiguous():
            raise ValueError("seq does not match the allocated layout")
        if status is not None and (status.dtype != torch.int32 or status.numel() < 1 or not status.is_cuda):
            raise ValueError("status must be a device int32 tensor")
        out = self.outputs()
        rc = lib().wt_build_noalloc(_ptr(seq), self.n, self.sigma, self.sym_bytes, ctypes.byref(out),
                                    _ptr(status), _stream(stream))
        _check(rc, "wt_build_noalloc")
        return self

    def status(self, stream=None) -> int:
        return int(lib().wt_status_get(_ptr(self.scratch), _stream(stream)))

    # -- queries ------------------------------------------------------------
    def _need_dirs(self):
        if self.rank is None:
            raise ValueError("queries need a tree built with directories")

    def access(self, i: torch.Tensor, stream=None) -> torch.Tensor:
        self._need_dirs()
        i = i.to(torch.int64).contiguous()
        out = torch.empty(i.numel(), dtype=torch.int32, device=i.device)
        v = self.view()
        _check(lib().wt_access(ctypes.byref(v), _ptr(i), i.numel(), _ptr(out), _stream(stream)), "wt_access")
        return out

    def rank_query(self, c: torch.Tensor, i: torch.Tensor, stream=None) -> torch.Tensor:
        self._need_dirs()
        c = c.to(torch.int32).contiguous()
        i = i.to(torch.int64).contiguous()
        out = torch.empty(i.numel(), dtype=torch.int64, device=i.device)
        v = self.view()
        _check(lib().wt_rank(ctypes.byref(v), _ptr(c), _ptr(i), i.numel(), _ptr(out), _stream(stream)), "wt_rank")
        return out

    def select_query(self, c: torch.Tensor, k: torch.Tensor, stream=None) -> torch.Tensor:
        self._need_dirs()
        c = c.to(torch.int32).contiguous()
        k = k.to(torch.int64).contiguous()
        out = torch.empty(k.numel(), dtype=torch.int64, device=k.device)
        v = self.view()
        _check(lib().wt_select(ctypes.byref(v), _ptr(c), _ptr(k), k.numel(), _ptr(out), _stream(stream)),
               "wt_select")
        return out

    def to_numpy(self) -> dict:
        import numpy as np
        u = lambda t: None if t is None else t.cpu().numpy().view(np.uint64)
        return {"L": self.L, "n": self.n, "sigma": self.sigma, "bits": u(self.bits), "C": u(self.C),
                "rank": u(self.rank), "sel1": u(self.sel1), "sel0": u(self.sel0), "sel_counts": u(self.sel_counts)}


@dataclass
class WaveletMatrix:
    """Device buffers of one built wavelet matrix: the tree's buffers plus the
    per-level zero counts (C is produced too; the queries do not use it)."""
    tree: WaveletTree
    zeros: torch.Tensor

    @staticmethod
    def allocate(n: int, sigma: int, sym_bytes: int, directories: bool = True, device="cuda") -> "WaveletMatrix":
        t = WaveletTree.allocate(n, sigma, sym_bytes, directories, device)
        return WaveletMatrix(t, torch.empty(max(t.L, 1), dtype=torch.int64, device=device))

    @property
    def L(self) -> int:
        return self.tree.L

    @property
    def n(self) -> int:
        return self.tree.n

    def build_from(self, seq: torch.Tensor, stream=None) -> "WaveletMatrix":
        """Launch wt_build_matrix on ``seq`` into this matrix's buffers (asynchronous)."""
        t = self.tree
        if not seq.is_cuda or seq.element_size() != t.sym_bytes or seq.numel() != t.n or not seq.is_contiguous():
            raise ValueError("seq does not match the allocated layout")
        out = t.outputs()
        rc = lib().wt_build_matrix(_ptr(seq), t.n, t.sigma, t.sym_bytes, ctypes.byref(out), _ptr(self.zeros),
                                   _ptr(t.scratch), t.scratch.numel(), _stream(stream))
        _check(rc, "wt_build_matrix")
        return self

    def status(self, stream=None) -> int:
        return self.tree.status(stream)

    def view(self) -> MatrixView:
        t = self.tree
        return MatrixView(_ptr(t.bits), _ptr(self.zeros), _ptr(t.rank), _ptr(t.sel1), _ptr(t.sel0),
                          _ptr(t.sel_counts), t.n, t.sigma, t.L)

    def access(self, i: torch.Tensor, stream=None) -> torch.Tensor:
        self.tree._need_dirs()
        i = i.to(torch.int64).contiguous()
        out = torch.empty(i.numel(), dtype=torch.int32, device=i.device)
        v = self.view()
        _check(lib().wt_matrix_access(ctypes.byref(v), _ptr(i), i.numel(), _ptr(out), _stream(stream)),
               "wt_matrix_access")
        return out

    def rank_query(self, c: torch.Tensor, i: torch.Tensor, stream=None) -> torch.Tensor:
        self.tree._need_dirs()
        c = c.to(torch.int32).contiguous()
        i = i.to(torch.int64).contiguous()
        out = torch.empty(i.numel(), dtype=torch.int64, device=i.device)
        v = self.view()
        _check(lib().wt_matrix_rank(ctypes.byref(v), _ptr(c), _ptr(i), i.numel(), _ptr(out), _stream(stream)),
               "wt_matrix_rank")
        return out

    def select_query(self, c: torch.Tensor, k: torch.Tensor, stream=None) -> torch.Tensor:
        self.tree._need_dirs()
        c = c.to(torch.int32).contiguous()
        k = k.to(torch.int64).contiguous()
        out = torch.empty(k.numel(), dtype=torch.int64, device=k.device)
        v = self.view()
        _check(lib().wt_matrix_select(ctypes.byref(v), _ptr(c), _ptr(k), k.numel(), _ptr(out), _stream(stream)),
               "wt_matrix_select")
        return out

    def to_numpy(self) -> dict:
        import numpy as np
        d = self.tree.to_numpy()
        d["zeros"] = self.zeros.cpu().numpy().view(np.uint64)[: self.L]
        return d


def build_matrix(seq: torch.Tensor, sigma: int, directories: bool = True, stream=None) -> WaveletMatrix:
    """Allocate buffers and build the wavelet matrix of ``seq``."""
    m = WaveletMatrix.allocate(seq.numel(), sigma, seq.element_size(), directories, seq.device)
    return m.build_from(seq, stream)


@dataclass
class WaveletMultiary:
    """Device buffers of one 4-ary wavelet tree (byte symbols): per level the
    2-bit entries, C, and the digit directories (int64 tensors hold uint64)."""
    n: int
    sigma: int
    Lq: int
    digits: torch.Tensor
    C: torch.Tensor
    rank4: torch.Tensor
    sel4: torch.Tensor
    counts4: torch.Tensor
    scratch: torch.Tensor

    @staticmethod
    def allocate(n: int, sigma: int, device="cuda") -> "WaveletMultiary":
        lay = plan(n, sigma, 1)
        Lq = (lay.L + 1) // 2
        R = lay.rank_len
        e = lambda *shape: torch.empty(*shape, dtype=torch.int64, device=device)
        return WaveletMultiary(n=n, sigma=sigma, Lq=Lq, digits=e(Lq, (n + 31) // 32), C=e(sigma + 1),
                               rank4=e(Lq, R, 4), sel4=e(Lq, 4, lay.sel_cap), counts4=e(Lq, 4),
                               scratch=torch.empty(max(lay.scratch_bytes, 256), dtype=torch.uint8, device=device))

    def build_from(self, seq: torch.Tensor, stream=None) -> "WaveletMultiary":
        if not seq.is_cuda or seq.element_size() != 1 or seq.numel() != self.n or not seq.is_contiguous():
            raise ValueError("seq must be a contiguous device tensor of n byte symbols")
        out = MultiaryOutputs(_ptr(self.digits), _ptr(self.C), _ptr(self.rank4), _ptr(self.sel4),
                              _ptr(self.counts4))
        rc = lib().wt_build_multiary(_ptr(seq), self.n, self.sigma, 1, ctypes.byref(out), _ptr(self.scratch),
                                     self.scratch.numel(), _stream(stream))
        _check(rc, "wt_build_multiary")
        return self

    def status(self, stream=None) -> int:
        return int(lib().wt_status_get(_ptr(self.scratch), _stream(stream)))

    def view(self) -> MultiaryView:
        return MultiaryView(_ptr(self.digits), _ptr(self.C), _ptr(self.rank4), _ptr(self.sel4), _ptr(self.counts4),
                            self.n, self.sigma, self.Lq)

    def access(self, i: torch.Tensor, stream=None) -> torch.Tensor:
        i = i.to(torch.int64).contiguous()
        out = torch.empty(i.numel(), dtype=torch.int32, device=i.device)
        v = self.view()
        _check(lib().wt_multiary_access(ctypes.byref(v), _ptr(i), i.numel(), _ptr(out), _stream(stream)),
               "wt_multiary_access")
        return out

    def rank_query(self, c: torch.Tensor, i: torch.Tensor, stream=None) -> torch.Tensor:
        c = c.to(torch.int32).contiguous()
        i = i.to(torch.int64).contiguous()
        out = torch.empty(i.numel(), dtype=torch.int64, device=i.device)
        v = self.view()
        _check(lib().wt_multiary_rank(ctypes.byref(v), _ptr(c), _ptr(i), i.numel(), _ptr(out), _stream(stream)),
               "wt_multiary_rank")
        return out

    def select_query(self, c: torch.Tensor, k: torch.Tensor, stream=None) -> torch.Tensor:
        c = c.to(torch.int32).contiguous()
        k = k.to(torch.int64).contiguous()
        out = torch.empty(k.numel(), dtype=torch.int64, device=k.device)
        v = self.view()
        _check(lib().wt_multiary_select(ctypes.byref(v), _ptr(c), _ptr(k), k.numel(), _ptr(out), _stream(stream)),
               "wt_multiary_select")
        return out

    def to_numpy(self) -> dict:
        import numpy as np
        u = lambda t: t.cpu().numpy().view(np.uint64)
        return {"Lq": self.Lq, "n": self.n, "sigma": self.sigma, "digits": u(self.digits), "C": u(self.C),
                "rank4": u(self.rank4), "sel4": u(self.sel4), "counts4": u(self.counts4)}


def build_multiary(seq: torch.Tensor, sigma: int, stream=None) -> WaveletMultiary:
    """Allocate buffers and build the 4-ary wavelet tree of ``seq`` (byte symbols)."""
    return WaveletMultiary.allocate(seq.numel(), sigma, seq.device).build_from(seq, stream)


def build(seq: torch.Tensor, sigma: int, directories: bool = True, stream=None) -> WaveletTree:
    """Allocate buffers and build the tree of ``seq`` (1-, 2- or 4-byte symbols)."""
    t = WaveletTree.allocate(seq.numel(), sigma, seq.element_size(), directories, seq.device)
    return t.build_from(seq, stream)


def batch_plan(jobs) -> BatchLayout:
    arr = (Job * max(len(jobs), 1))(*jobs)
    lay = BatchLayout()
    _check(lib().wt_batch_plan(arr, len(jobs), ctypes.byref(lay)), "wt_batch_plan")
    return lay


class Batch:
    """Many sequences built together by wt_batch_run (one persistent launch
    of the work kernel, or one launch per phase).  All outputs live in one
    int64 slab (each buffer 256-byte aligned); ``trees[i]`` views job i."""

    def __init__(self, seqs: list[torch.Tensor], sigmas: list[int], stream=None):
        if len(seqs) != len(sigmas):
            raise ValueError("one sigma per sequence")
        dev = seqs[0].device if seqs else torch.device("cuda")
        shapes, total = [], 0
        for q, sigma in zip(seqs, sigmas):
            if not q.is_cuda or not q.is_contiguous() or q.data_ptr() % 16:
                raise ValueError("sequences must be contiguous, 16-byte aligned device tensors")
            lay, sh = WaveletTree.output_words(q.numel(), int(sigma), q.element_size())
            offs = []
            for shape in sh:
                offs.append(total)
                words = 1
                for d in shape:
                    words *= d
                total += -(-words // 32) * 32
            shapes.append((lay, sh, offs))
        self.slab = torch.empty(max(total, 32), dtype=torch.int64, device=dev)
        self.trees: list[WaveletTree] = []
        jobs = []
        for q, sigma, (lay, sh, offs) in zip(seqs, sigmas, shapes):
            views = []
            for shape, off in zip(sh, offs):
                words = 1
                for d in shape:
                    words *= d
                views.append(self.slab[off:off + words].view(*shape))
            t = WaveletTree(n=q.numel(), sigma=int(sigma), L=lay.L, sym_bytes=q.element_size(), bits=views[0],
                            C=views[1], rank=views[2], sel1=views[3], sel0=views[4], sel_counts=views[5],
                            scratch=self.slab[:0], layout=lay)
            self.trees.append(t)
            jobs.append(Job(_ptr(q), q.numel(), int(sigma), q.element_size(), 0, t.outputs()))
        self.seqs = list(seqs)
        self.jobs = (Job * max(len(jobs), 1))(*jobs)
        self.njobs = len(jobs)
        self.layout = BatchLayout()
        _check(lib().wt_batch_plan(self.jobs, self.njobs, ctypes.byref(self.layout)), "wt_batch_plan")
        self.scratch = torch.empty(max(self.layout.scratch_bytes, 256), dtype=torch.uint8, device=dev)
        rc = lib().wt_batch_prepare(self.jobs, self.njobs, ctypes.byref(self.layout), _ptr(self.scratch),
                                    self.scratch.numel(), _stream(stream))
        _check(rc, "wt_batch_prepare")

    def run(self, tune: Tune | None = None, stream=None) -> "Batch":
        t = tune if tune is not None else Tune()
        _check(lib().wt_batch_run(ctypes.byref(self.layout), ctypes.byref(t), _ptr(self.scratch), _stream(stream)),
               "wt_batch_run")
        return self

    def status(self, stream=None) -> tuple[int, list[int]]:
        codes = (ctypes.c_int32 * max(self.njobs, 1))()
        rc = lib().wt_batch_status(ctypes.byref(self.layout), _ptr(self.scratch), codes, _stream(stream))
        return int(rc), [int(codes[i]) for i in range(self.njobs)]


def views_tensor(trees: list, device="cuda") -> torch.Tensor:
    """Device array of wt_view for `trees` (a uint8 tensor holding the structs)."""
    arr = (View * max(len(trees), 1))(*[t.view() for t in trees])
    host = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
    return host.to(device)


def query_multi(views: torch.Tensor, ntrees: int, tree: torch.Tensor, kind: torch.Tensor, a: torch.Tensor,
                b: torch.Tensor, stream=None) -> torch.Tensor:
    """Mixed access/rank/select over many trees (wt_query_multi); int64 answers."""
    tree = tree.to(torch.int32).contiguous()
    kind = kind.to(torch.uint8).contiguous()
    a = a.to(torch.int64).contiguous()
    b = b.to(torch.int64).contiguous()
    out = torch.empty(tree.numel(), dtype=torch.int64, device=tree.device)
    _check(lib().wt_query_multi(_ptr(views), ntrees, _ptr(tree), _ptr(kind), _ptr(a), _ptr(b), tree.numel(),
                                _ptr(out), _stream(stream)), "wt_query_multi")
    return out


def build_rank_select(bits: torch.Tensor, n: int, L: int, stream=None) -> dict:
    """Standalone directories of level bitmaps ``bits`` (L, ceil(n/64)) int64."""
    rank_len = (n + RANK_BLOCK_BITS - 1) // RANK_BLOCK_BITS + 1
    cap = (n + SELECT_SAMPLE - 1) // SELECT_SAMPLE + 1
    dev = bits.device
    e = lambda *shape: torch.empty(*shape, dtype=torch.int64, device=dev)
    rank, sel1, sel0, counts = e(L, rank_len), e(L, cap), e(L, cap), e(2 * L)
    sbytes = int(lib().wt_rank_select_scratch_bytes(n, L))
    scratch = torch.empty(max(sbytes, 256), dtype=torch.uint8, device=dev)
    rc = lib().wt_build_rank_select(_ptr(bits.contiguous()), n, L, _ptr(rank), _ptr(sel1), _ptr(sel0),
                                    _ptr(counts), _ptr(scratch), scratch.numel(), _stream(stream))
    _check(rc, "wt_build_rank_select")
    return {"rank": rank, "sel1": sel1, "sel0": sel0, "sel_counts": counts, "_scratch": scratch}


def set_fused_levels(levels):
    """0/False: no fused levels; 1/True: from the first level whose nodes fit;
    m >= 2: at most the last m levels (this host thread's later launches)."""
    _check(lib().wt_set_fused_levels(int(levels)), "wt_set_fused_levels")


def histogram_path(n: int, sigma: int, sym_bytes: int) -> int:
    """Which histogram wt_build runs for these sizes (HIST_*), under this thread's settings."""
    rc = lib().wt_histogram_path(n, sigma, sym_bytes)
    if rc < 0:
        raise WTError(rc, "wt_histogram_path")
    return rc


def set_sliced_histogram(on: bool):
    _check(lib().wt_set_sliced_histogram(1 if on else 0), "wt_set_sliced_histogram")


def set_level_pairs(on: bool) -> bool:
    """Two levels per pass for byte alphabets on or off; returns the previous setting."""
    return lib().wt_set_level_pairs(1 if on else 0) != 0


def set_lookback_spin_limit(polls: int):
    _check(lib().wt_set_lookback_spin_limit(polls), "wt_set_lookback_spin_limit")


def timing_enable(on: bool = True):
    _check(lib().wt_timing_enable(1 if on else 0), "wt_timing_enable")


def timing_collect(cap: int = 1 << 16) -> list[float]:
    buf = (ctypes.c_float * cap)()
    rc = lib().wt_timing_collect(buf, cap)
    if rc < 0:
        raise WTError(rc, "wt_timing_collect")
    return [float(buf[i]) for i in range(min(rc, cap))]


def to_device(S, device="cuda") -> torch.Tensor:
    """numpy symbols (uint8/uint16/uint32) -> device tensor of the same width."""
    import numpy as np
    raw = {1: np.int8, 2: np.int16, 4: np.int32}[S.dtype.itemsize]
    return torch.from_numpy(np.ascontiguousarray(S).view(raw)).to(device)


@dataclass
class WaveletHuffman:
    """Device buffers of one Huffman-shaped wavelet tree (byte symbols),
    sized for the largest height the input length allows (int64 tensors hold
    uint64; lens is int32)."""
    n: int
    sigma: int
    h_cap: int
    bits: torch.Tensor
    C: torch.Tensor
    rank: torch.Tensor
    sel1: torch.Tensor
    sel0: torch.Tensor
    sel_counts: torch.Tensor
    lens: torch.Tensor
    codes: torch.Tensor
    nd: torch.Tensor
    tables: torch.Tensor
    scratch: torch.Tensor
    h: int = 0

    @staticmethod
    def allocate(n: int, sigma: int, device="cuda", h_cap: int | None = None) -> "WaveletHuffman":
        L = lib()
        hb, sb, tb = ctypes.c_uint32(0), ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(L.wt_huffman_plan(n, sigma, 0, ctypes.byref(hb), None, None), "wt_huffman_plan")
        cap = hb.value if h_cap is None else h_cap
        _check(L.wt_huffman_plan(n, sigma, cap, None, ctypes.byref(sb), ctypes.byref(tb)), "wt_huffman_plan")
        lay = plan(n, sigma, 1)
        e = lambda *shape: torch.empty(*shape, dtype=torch.int64, device=device)
        k = max(cap, 1)
        return WaveletHuffman(n=n, sigma=sigma, h_cap=cap, bits=e(k, lay.words_per_level), C=e(sigma + 1),
                              rank=e(k, lay.rank_len), sel1=e(k, lay.sel_cap), sel0=e(k, lay.sel_cap),
                              sel_counts=e(2 * k), lens=torch.empty(256, dtype=torch.int32, device=device),
                              codes=e(256), nd=e(k), tables=torch.empty(tb.value, dtype=torch.uint8, device=device),
                              scratch=torch.empty(max(sb.value, 256), dtype=torch.uint8, device=device))

    def build_from(self, seq: torch.Tensor, stream=None) -> "WaveletHuffman":
        if not seq.is_cuda or seq.element_size() != 1 or seq.numel() != self.n or not seq.is_contiguous():
            raise ValueError("seq must be a contiguous device tensor of n byte symbols")
        out = HuffmanOutputs(_ptr(self.bits), _ptr(self.C), _ptr(self.rank), _ptr(self.sel1), _ptr(self.sel0),
                             _ptr(self.sel_counts), _ptr(self.lens), _ptr(self.codes), _ptr(self.nd),
                             _ptr(self.tables))
        h = ctypes.c_uint32(0)
        rc = lib().wt_build_huffman(_ptr(seq), self.n, self.sigma, ctypes.byref(out), self.h_cap, ctypes.byref(h),
                                    _ptr(self.scratch), self.scratch.numel(), _stream(stream))
        _check(rc, "wt_build_huffman")
        self.h = int(h.value)
        return self

    def status(self, stream=None) -> int:
        return int(lib().wt_status_get(_ptr(self.scratch), _stream(stream)))

    def view(self) -> HuffmanView:
        return HuffmanView(_ptr(self.bits), _ptr(self.rank), _ptr(self.sel1), _ptr(self.sel0), _ptr(self.tables),
                           self.n, self.sigma, self.h)

    def access(self, i: torch.Tensor, stream=None) -> torch.Tensor:
        i = i.to(torch.int64).contiguous()
        out = torch.empty(i.numel(), dtype=torch.int32, device=i.device)
        v = self.view()
        _check(lib().wt_huffman_access(ctypes.byref(v), _ptr(i), i.numel(), _ptr(out), _stream(stream)),
               "wt_huffman_access")
        return out

    def rank_query(self, c: torch.Tensor, i: torch.Tensor, stream=None) -> torch.Tensor:
        c = c.to(torch.int32).contiguous()
        i = i.to(torch.int64).contiguous()
        out = torch.empty(i.numel(), dtype=torch.int64, device=i.device)
        v = self.view()
        _check(lib().wt_huffman_rank(ctypes.byref(v), _ptr(c), _ptr(i), i.numel(), _ptr(out), _stream(stream)),
               "wt_huffman_rank")
        return out

    def select_query(self, c: torch.Tensor, k: torch.Tensor, stream=None) -> torch.Tensor:
        c = c.to(torch.int32).contiguous()
        k = k.to(torch.int64).contiguous()
        out = torch.empty(k.numel(), dtype=torch.int64, device=k.device)
        v = self.view()
        _check(lib().wt_huffman_select(ctypes.byref(v), _ptr(c), _ptr(k), k.numel(), _ptr(out), _stream(stream)),
               "wt_huffman_select")
        return out

    def to_numpy(self) -> dict:
        import numpy as np
        u = lambda t: t.cpu().numpy().view(np.uint64)
        h = self.h
        counts = u(self.sel_counts)
        return {"h": h, "n": self.n, "sigma": self.sigma, "bits": u(self.bits)[:h], "C": u(self.C),
                "rank": u(self.rank)[:h], "sel1": u(self.sel1)[:h], "sel0": u(self.sel0)[:h],
                "sel_counts": counts[: 2 * h], "lens": self.lens.cpu().numpy().view(np.uint32),
                "codes": u(self.codes), "nd": u(self.nd)[:h]}


def build_huffman(seq: torch.Tensor, sigma: int, stream=None) -> WaveletHuffman:
    """Allocate buffers and build the Huffman-shaped wavelet tree of ``seq`` (byte symbols)."""
    return WaveletHuffman.allocate(seq.numel(), sigma, seq.device).build_from(seq, stream)


def build_sort(seq: torch.Tensor, sigma: int, stream=None, tree: WaveletTree | None = None) -> WaveletTree:
    """Build the tree of ``seq`` (byte symbols) by sortWT (wt_build_sort): the
    same outputs as ``build`` with directories, from the sorted copies of S
    instead of the level passes.  ``tree``, when given, is reused (its
    scratch grown to the sortWT size)."""
    n = seq.numel()
    if not seq.is_cuda or seq.element_size() != 1 or not seq.is_contiguous():
        raise ValueError("seq must be a contiguous device tensor of byte symbols")
    nbytes = int(lib().wt_sort_scratch_bytes(n, sigma))
    if nbytes == 0:
        raise WTError(WT_ERR_RANGE, "wt_sort_scratch_bytes")
    t = tree if tree is not None else WaveletTree.allocate(n, sigma, 1, True, seq.device)
    if t.scratch.numel() < nbytes:
        t.scratch = torch.empty(nbytes, dtype=torch.uint8, device=seq.device)
    out = Outputs(_ptr(t.bits), _ptr(t.C), _ptr(t.rank), _ptr(t.sel1), _ptr(t.sel0), _ptr(t.sel_counts))
    _check(lib().wt_build_sort(_ptr(seq), n, sigma, 1, ctypes.byref(out), _ptr(t.scratch), t.scratch.numel(),
                               _stream(stream)), "wt_build_sort")
    return t

