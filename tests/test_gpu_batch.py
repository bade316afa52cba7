"""GPU parity of the batched build (wt_batch_run): every job's buffers equal
the oracle's bit for bit (and wt_build's), in both launch forms, under
several launch tunables, inside a captured graph, and again after the
inputs change.  Integer work throughout: the tolerance is zero."""
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


def assert_same(got: dict, want: dict, ctx: str):
    for k in KEYS:
        g = np.asarray(got[k], dtype=np.uint64).reshape(-1)
        w = np.asarray(want[k], dtype=np.uint64).reshape(-1)
        assert g.shape == w.shape, (ctx, k, g.shape, w.shape)
        if not np.array_equal(g, w):
            bad = np.flatnonzero(g != w)
            raise AssertionError(f"{ctx}: {k} differs at {bad.size} of {g.size}, first {bad[:5]}: "
                                 f"got {g[bad[:5]]} want {w[bad[:5]]}")


def mixed_jobs(seed=11):
    """Edge sizes and every width pairing the level pass has."""
    rng = np.random.default_rng(seed)
    spec = [(0, 4), (1, 1), (1, 2), (5, 1), (63, 3), (64, 256), (65, 5), (4095, 256), (4096, 2), (4097, 17),
            (16383, 256), (16384, 256), (16385, 256), (40000, 4), (70001, 256), (9000, 257), (8192, 1 << 16),
            (8193, 1 << 16), (30000, 1000), (5000, 1 << 20), (12289, (1 << 16) + 1), (3, 1 << 20), (131072, 256),
            (100000, 65536), (2, 2), (777, 1 << 12)]
    out = []
    for n, sigma in spec:
        S = rng.integers(0, sigma, n, dtype=np.uint64).astype(inputs.dtype_for_sigma(sigma))
        out.append((S, sigma))
    # a u32 input with a small alphabet (narrowed to bytes after level 0)
    out.append((rng.integers(0, 200, 20000).astype(np.uint32), 200))
    # u16 input with sigma <= 256
    out.append((rng.integers(0, 100, 33333).astype(np.uint16), 100))
    # whole-job histogram (5120 <= sigma <= 2^16) from a u32 input
    out.append((rng.integers(0, 40000, 20000).astype(np.uint32), 40000))
    # whole-job histogram with one symbol far past 2^15 occurrences (its
    # packed LDS counter hands 2^15 to the global count many times)
    heavy = np.where(rng.random(150001) < 0.8, 7, rng.integers(0, 6000, 150001)).astype(np.uint16)
    out.append((heavy, 6000))
    return out


def make_batch(wt, jobs):
    seqs = [wt.to_device(S) for S, _ in jobs]
    return wt.Batch(seqs, [s for _, s in jobs]), seqs


def check_batch(wt, oracle_mod, b, jobs, ctx):
    rc, codes = b.status()
    assert rc == wt.WT_OK, (ctx, rc, codes)
    for i, ((S, sigma), t) in enumerate(zip(jobs, b.trees)):
        assert_same(t.to_numpy(), oracle_mod.build_all(S, sigma), f"{ctx} job {i} n={S.size} sigma={sigma}")


@pytest.mark.parametrize("mode", ["persistent", "per_phase"])
def test_batch_mixed_matches_oracle(wtmod, oracle_mod, mode):
    jobs = mixed_jobs()
    say(f"[batch] mixed {len(jobs)} jobs, {mode}")
    b, _ = make_batch(wtmod, jobs)
    tune = wtmod.Tune(mode=wtmod.BATCH_PERSISTENT if mode == "persistent" else wtmod.BATCH_PER_PHASE)
    b.run(tune)
    torch.cuda.synchronize()
    check_batch(wtmod, oracle_mod, b, jobs, mode)


@pytest.mark.parametrize("tune", [dict(chunk=4), dict(blocks_per_cu=1), dict(blocks_per_cu=1, chunk=16),
                                  dict(mode=1, chunk=8, blocks_per_cu=2)])
def test_batch_tunes_identical(wtmod, oracle_mod, tune):
    jobs = mixed_jobs(seed=12)
    say(f"[batch] tune {tune}")
    b, _ = make_batch(wtmod, jobs)
    b.run(wtmod.Tune(**tune))
    torch.cuda.synchronize()
    check_batch(wtmod, oracle_mod, b, jobs, f"tune {tune}")


def test_batch_config4_shape_matches_single_builds(wtmod, oracle_mod):
    """The batched-build recipe (lengths log-uniform, sigma in {4, 256, 2^16})
    at 192 sequences up to 2^17: every job equals wt_build's output, and a
    sample of jobs equals the oracle."""
    seqs = inputs.batch(count=192, lo_exp=10.0, hi_exp=17.0)
    jobs = [(q.S, q.sigma) for q in seqs]
    say(f"[batch] config-4 shape, {len(jobs)} jobs, {sum(S.size for S, _ in jobs)} symbols")
    b, dev = make_batch(wtmod, jobs)
    b.run()
    torch.cuda.synchronize()
    rc, codes = b.status()
    assert rc == wtmod.WT_OK, codes
    for i, ((S, sigma), q) in enumerate(zip(jobs, dev)):
        single = wtmod.build(q, sigma)
        torch.cuda.synchronize()
        assert_same(b.trees[i].to_numpy(), single.to_numpy(), f"job {i} vs wt_build")
    for i in range(0, len(jobs), 16):
        S, sigma = jobs[i]
        assert_same(b.trees[i].to_numpy(), oracle_mod.build_all(S, sigma), f"job {i} vs oracle")


def test_batch_graph_replay(wtmod, oracle_mod):
    """wt_batch_run captured in a graph: every replay equals the eager run,
    with eager work and synchronisation between replays."""
    jobs = mixed_jobs(seed=13)
    b, _ = make_batch(wtmod, jobs)
    b.run()
    torch.cuda.synchronize()
    want = [t.to_numpy() for t in b.trees]
    check_batch(wtmod, oracle_mod, b, jobs, "eager")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        b.run(stream=s)  # warm-up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            b.run(stream=s)
    torch.cuda.synchronize()
    for r in range(3):
        b.slab.fill_(-1)  # outputs wiped: the replay must rewrite every word
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        say(f"[batch] graph replay {r}")
        assert b.status()[0] == wtmod.WT_OK
        for i, t in enumerate(b.trees):
            assert_same(t.to_numpy(), want[i], f"replay {r} job {i}")


def test_batch_rerun_after_input_change(wtmod, oracle_mod):
    jobs = mixed_jobs(seed=14)
    b, dev = make_batch(wtmod, jobs)
    b.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(99)
    new = []
    for (S, sigma), q in zip(jobs, dev):
        S2 = rng.integers(0, sigma, S.size, dtype=np.uint64).astype(S.dtype)
        q.copy_(wtmod.to_device(S2))
        new.append((S2, sigma))
    b.run()
    torch.cuda.synchronize()
    check_batch(wtmod, oracle_mod, b, new, "rerun")


def test_batch_symbol_error_is_per_job(wtmod, oracle_mod):
    jobs = mixed_jobs(seed=15)
    bad = 9
    S, sigma = jobs[bad]
    assert (S.size, sigma, S.dtype) == (4097, 17, np.uint8)
    S = S.copy()
    S[1234] = 200
    jobs[bad] = (S, sigma)
    b, _ = make_batch(wtmod, jobs)
    b.run()
    torch.cuda.synchronize()
    rc, codes = b.status()
    assert rc == wtmod.WT_ERR_SYMBOL
    assert codes[bad] == wtmod.WT_ERR_SYMBOL
    assert all(c == wtmod.WT_OK for i, c in enumerate(codes) if i != bad)
    for i, ((S, sigma), t) in enumerate(zip(jobs, b.trees)):
        if i != bad:
            assert_same(t.to_numpy(), oracle_mod.build_all(S, sigma), f"job {i} beside a rejected job")


def test_batch_bounded_wait_gives_up_cleanly(wtmod, oracle_mod):
    """spin_limit=1: a block that finds its level not ready gives up at once
    (the abort path; every wave still exits).  The run reports either success
    with correct outputs or WT_ERR_TIMEOUT; a normal run afterwards on the
    same scratch is correct again."""
    jobs = mixed_jobs(seed=16)
    b, _ = make_batch(wtmod, jobs)
    b.run(wtmod.Tune(spin_limit=1))
    torch.cuda.synchronize()
    rc, codes = b.status()
    say(f"[batch] spin_limit=1 -> {rc}")
    assert rc in (wtmod.WT_OK, wtmod.WT_ERR_TIMEOUT)
    if rc == wtmod.WT_OK:
        check_batch(wtmod, oracle_mod, b, jobs, "spin_limit=1")
    b.run()
    torch.cuda.synchronize()
    check_batch(wtmod, oracle_mod, b, jobs, "after timeout")


def test_batch_empty_and_single(wtmod, oracle_mod):
    b, _ = make_batch(wtmod, [(np.zeros(0, np.uint8), 3)])
    b.run()
    torch.cuda.synchronize()
    check_batch(wtmod, oracle_mod, b, [(np.zeros(0, np.uint8), 3)], "n=0 only")
    S = inputs.text_like(300000)
    b, _ = make_batch(wtmod, [(S, 256)])
    b.run(wtmod.Tune(mode=wtmod.BATCH_PER_PHASE))
    torch.cuda.synchronize()
    check_batch(wtmod, oracle_mod, b, [(S, 256)], "single text job")


@pytest.mark.parametrize("levels", [0, 3, 1])
def test_batch_fused_levels_setting(wtmod, oracle_mod, levels):
    """No fused levels, at most the last three, or all that fit: the same
    buffers as the oracle's in every case."""
    jobs = mixed_jobs(seed=14)
    say(f"[batch] fused levels setting {levels}")
    b, _ = make_batch(wtmod, jobs)
    try:
        wtmod.set_fused_levels(levels)
        b.run(wtmod.Tune(mode=wtmod.BATCH_PER_PHASE))
        torch.cuda.synchronize()
    finally:
        wtmod.set_fused_levels(1)
    check_batch(wtmod, oracle_mod, b, jobs, f"fused levels {levels}")
