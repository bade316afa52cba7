"""Kernel timing mode (wt_timing_enable / wt_timing_collect): every level-pass
launch carries its own start and stop events.  A timed build must equal an
untimed one bit for bit, and it must report one positive duration per level
pass, in launch order."""
import math
import sys

import numpy as np
import pytest

from paper_1407_8142_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BUFS = ("bits", "C", "rank", "sel1", "sel0", "sel_counts")


@pytest.fixture(scope="module")
def wtmod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1407_8142_amd import wt
    wt.lib()
    return wt


def timed(wtmod, fn):
    wtmod.timing_collect()
    wtmod.timing_enable(True)
    try:
        out = fn()
        torch.cuda.synchronize()
    finally:
        wtmod.timing_enable(False)
    return out, wtmod.timing_collect()


def check_times(ms, count):
    assert len(ms) == count
    assert all(math.isfinite(x) and 0.0 < x < 1000.0 for x in ms), ms


@pytest.mark.parametrize("n,sigma,dtype", [(3 * (1 << 20) + 77, 256, np.uint8), (200001, 1000, np.uint32),
                                           ((1 << 20) + 5, 1 << 16, np.uint16), (70000, 5, np.uint8)])
def test_timed_tree_equals_untimed(wtmod, n, sigma, dtype):
    print(f"[timing] tree n={n} sigma={sigma} {np.dtype(dtype).name}", flush=True)
    sys.stdout.flush()
    rng = np.random.default_rng(n ^ sigma)
    S = rng.integers(0, sigma, n).astype(dtype)
    d = wtmod.to_device(S)
    ref = wtmod.build(d, sigma)
    t, ms = timed(wtmod, lambda: wtmod.build(d, sigma))
    assert t.status() == wtmod.WT_OK
    L = max(1, (sigma - 1).bit_length())
    check_times(ms, L)
    for k in BUFS:
        assert torch.equal(getattr(t, k), getattr(ref, k)), k


def test_timed_matrix_and_huffman(wtmod):
    print("[timing] matrix and Huffman, text-like n=2^21", flush=True)
    S = inputs.text_like(1 << 21, 256, index=5)
    d = wtmod.to_device(S)
    m0 = wtmod.build_matrix(d, 256)
    m, ms = timed(wtmod, lambda: wtmod.build_matrix(d, 256))
    check_times(ms, 8)
    for k in BUFS:
        assert torch.equal(getattr(m.tree, k), getattr(m0.tree, k)), k
    h0 = wtmod.build_huffman(d, 256)
    h, ms = timed(wtmod, lambda: wtmod.build_huffman(d, 256))
    got, ref = h.to_numpy(), h0.to_numpy()
    check_times(ms, int(ref["h"]))
    for k in ("bits", "rank", "C", "lens", "codes", "nd"):
        assert np.array_equal(got[k], ref[k]), k
