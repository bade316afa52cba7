"""wt_build_noalloc (the build whose scratch is the library's static device
array) against wt_build (caller scratch) on the same inputs: every output
buffer (bits, C, rank, sel1, sel0, sel_counts) equal bit for bit (integer
work: tolerance zero), on calls in a row whose later inputs are smaller and
of other widths (the array keeps the previous call's contents); a rejected
symbol reported through the status word and cleared by the next build; a
plan larger than the array refused before anything runs."""
import sys

import numpy as np
import pytest

from paper_1407_8142_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("bits", "C", "rank", "sel1", "sel0", "sel_counts")


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


def both(wt, S, sigma):
    d = wt.to_device(S)
    ref = wt.build(d, sigma)
    t = wt.WaveletTree.allocate(S.size, sigma, S.dtype.itemsize, True, d.device)
    for x in (t.bits, t.C, t.rank, t.sel1, t.sel0, t.sel_counts):
        x.fill_(-1)  # stale contents must not survive
    st = torch.full((1,), 12345, dtype=torch.int32, device=d.device)
    t.build_noalloc_from(d, st)
    torch.cuda.synchronize()
    assert ref.status() == wt.WT_OK
    return ref.to_numpy(), t.to_numpy(), int(st.item())


def assert_same(got, want, ctx):
    for k in KEYS:
        g = np.asarray(got[k], dtype=np.uint64).reshape(-1)
        w = np.asarray(want[k], dtype=np.uint64).reshape(-1)
        assert g.shape == w.shape, (ctx, k)
        bad = np.flatnonzero(g != w)
        assert bad.size == 0, f"{ctx}: {k} differs at {bad.size} of {g.size}, first {bad[:5]}"


def test_noalloc_equals_build_on_calls_in_a_row(wtmod):
    rng = np.random.default_rng(77)
    cases = [
        ("text-like u8 n=3000017", inputs.text_like(3_000_017), 256),
        ("u16 n=200003 sigma=40000", rng.integers(0, 40000, 200_003).astype(np.uint16), 40000),
        ("u32 n=70001 sigma=2^20+3", rng.integers(0, (1 << 20) + 3, 70_001).astype(np.uint32), (1 << 20) + 3),
        ("u8 n=4099 sigma=5", rng.integers(0, 5, 4099).astype(np.uint8), 5),
    ]
    for ctx, S, sigma in cases:
        say(f"[noalloc] {ctx}")
        assert wtmod.plan(S.size, sigma, S.dtype.itemsize).scratch_bytes <= wtmod.NOALLOC_SCRATCH_BYTES
        want, got, st = both(wtmod, S, sigma)
        assert st == wtmod.WT_OK, (ctx, st)
        assert_same(got, want, ctx)


def test_noalloc_status_word(wtmod):
    S = np.random.default_rng(3).integers(0, 100, 50_000).astype(np.uint8)
    S[777] = 200
    say("[noalloc] rejected symbol")
    d = wtmod.to_device(S)
    t = wtmod.WaveletTree.allocate(S.size, 100, 1, True, d.device)
    st = torch.zeros(1, dtype=torch.int32, device=d.device)
    t.build_noalloc_from(d, st)
    torch.cuda.synchronize()
    assert int(st.item()) == wtmod.WT_ERR_SYMBOL
    say("[noalloc] the next build clears it")
    S[777] = 5
    want, got, code = both(wtmod, S, 100)
    assert code == wtmod.WT_OK
    assert_same(got, want, "after a rejected build")


def test_noalloc_refuses_large_plans(wtmod):
    n = 80 << 20  # two 80 MiB sequence buffers
    assert wtmod.plan(n, 256, 1).scratch_bytes > wtmod.NOALLOC_SCRATCH_BYTES
    d = torch.zeros(n, dtype=torch.uint8, device="cuda")
    t = wtmod.WaveletTree.allocate(n, 256, 1, True, d.device)
    with pytest.raises(wtmod.WTError) as e:
        t.build_noalloc_from(d)
    assert e.value.rc == wtmod.WT_ERR_SCRATCH
