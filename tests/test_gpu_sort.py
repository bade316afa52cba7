"""GPU parity of sortWT (wt_build_sort), the second construction of the
tree: every output equals the oracle's bit for bit, and equals wt_build's
(the level passes) on the same input.  Integer work: tolerance zero."""
import sys

import numpy as np
import pytest

from paper_1407_8142_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("bits", "C", "rank", "sel1", "sel0", "sel_counts")
SIZES = [0, 1, 2, 63, 64, 65, 511, 512, 513, 4095, 4096, 4097, 16383, 16384, 16385, 69635, 200001]


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


def same(got, want, ctx):
    for k in KEYS:
        g = np.asarray(got[k], dtype=np.uint64).reshape(-1)
        w = np.asarray(want[k], dtype=np.uint64).reshape(-1)
        assert g.shape == w.shape, (ctx, k, g.shape, w.shape)
        if not np.array_equal(g, w):
            bad = np.flatnonzero(g != w)
            raise AssertionError(f"{ctx}: {k} differs at {bad.size} of {g.size}, first {bad[:5]}: "
                                 f"got {g[bad[:5]]} want {w[bad[:5]]}")


@pytest.mark.parametrize("sigma", [1, 2, 3, 5, 146, 256])
def test_sort_sizes(wtmod, oracle_mod, sigma):
    rng = np.random.default_rng(300 + sigma)
    for n in SIZES:
        S = rng.integers(0, sigma, n).astype(np.uint8)
        say(f"[sort] n={n} sigma={sigma}")
        t = wtmod.build_sort(wtmod.to_device(S), sigma)
        torch.cuda.synchronize()
        assert t.status() == wtmod.WT_OK
        same(t.to_numpy(), oracle_mod.build_all(S, sigma), f"n={n} sigma={sigma}")


@pytest.mark.parametrize("case", ["text", "sorted", "constant", "runs", "two_far", "zipf"])
def test_sort_equals_level_passes(wtmod, oracle_mod, case):
    rng = np.random.default_rng(17)
    n = 150001
    if case == "text":
        S, sigma = inputs.text_like(1 << 22), 256
    elif case == "sorted":
        S, sigma = np.sort(rng.integers(0, 256, n)).astype(np.uint8), 256
    elif case == "constant":
        S, sigma = np.full(n, 99, np.uint8), 128
    elif case == "runs":
        S, sigma = np.repeat(rng.integers(0, 256, 9000), rng.integers(1, 40, 9000)).astype(np.uint8), 256
    elif case == "two_far":
        S, sigma = np.where(rng.random(n) < 0.5, 0, 255).astype(np.uint8), 256
    else:
        S, sigma = (np.minimum(rng.zipf(1.2, n), 200) - 1).astype(np.uint8), 200
    say(f"[sort] {case}: n={S.size} sigma={sigma}")
    d = wtmod.to_device(S)
    a = wtmod.build_sort(d, sigma)
    b = wtmod.build(d, sigma)
    torch.cuda.synchronize()
    assert a.status() == wtmod.WT_OK and b.status() == wtmod.WT_OK
    same(a.to_numpy(), b.to_numpy(), case)
    if S.size <= 200001:
        same(a.to_numpy(), oracle_mod.build_all(S, sigma), case)


def test_sort_queries_use_the_tree_view(wtmod):
    S = np.random.default_rng(5).integers(0, 77, 30001).astype(np.uint8)
    t = wtmod.build_sort(wtmod.to_device(S), 77)
    i = torch.arange(0, S.size, 7, device="cuda")
    assert np.array_equal(t.access(i).cpu().numpy(), S[::7].astype(np.int32))


def test_sort_rejects_symbol(wtmod):
    S = np.random.default_rng(6).integers(0, 100, 50000).astype(np.uint8)
    S[123] = 200
    t = wtmod.build_sort(wtmod.to_device(S), 100)
    torch.cuda.synchronize()
    assert t.status() == wtmod.WT_ERR_SYMBOL
