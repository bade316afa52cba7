"""GPU test of the serving loop: requests arrive while others are building,
small ones are batched, trees are evicted under a tight HBM budget, and
query batches run against whatever is resident.  Every tree the server
kept equals the tree wt_build makes from the same input alone, and every
query answer equals naive counting over the input (bit for bit)."""
import sys

import numpy as np
import pytest

from paper_1407_8142_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1407_8142_amd import serve, wt
    wt.lib()
    return wt, serve


@pytest.mark.parametrize("h2d", [False, True], ids=["staged", "h2d"])
def test_serving_mix_equals_alone(mods, oracle_mod, h2d):
    """h2d: payloads in pinned host memory, copied after admission."""
    wt, serve = mods
    reqs, qtimes = inputs.serving_arrivals(0.05, rate=2000.0, qrate=120.0, n_exp=(10.0, 17.0), sigma_exp=(2.0, 20.0),
                                           index=7, max_requests=80)
    slab, layout, views = inputs.stage_requests(reqs)
    payloads = inputs.stage_pinned(slab, reqs, layout)[1] if h2d else views
    torch.cuda.synchronize()
    total = sum(sum(serve.Server.footprint(r.n, r.sigma, layout[i][1])) for i, r in enumerate(reqs))
    srv = serve.Server(budget_bytes=max(total // 3, 1 << 26), build_streams=3, small_n=1 << 14,
                       small_sigma=1 << 12)
    srv.keep_results = True
    issued = {}
    orig = srv.submit_queries

    def capture(qb):  # remember every batch's queries for checking
        issued[qb.qid] = qb
        orig(qb)

    srv.submit_queries = capture
    stats = serve.run_trace(srv, reqs, payloads, qtimes, slab, layout, qsize=3000, seed=3, select_share=0.3)
    torch.cuda.synchronize()
    print(f"[serve] built {stats.built} of {len(reqs)}, batches {stats.batches}, singles {stats.singles}, "
          f"evictions {stats.evictions}, query batches {len(stats.query_latency)}", flush=True)
    assert stats.failed == []
    assert stats.built == len(reqs)
    assert stats.batches > 0 and stats.singles > 0
    host = [v.cpu().numpy().view({1: np.uint8, 2: np.uint16, 4: np.uint32}[v.element_size()]) for v in views]
    # Trees kept resident: identical to a build of the same input alone.
    for rid in srv.resident_ids():
        alone = wt.build(views[rid], reqs[rid].sigma)
        torch.cuda.synchronize()
        got, want = srv.tree(rid).to_numpy(), alone.to_numpy()
        for k in ("bits", "C", "rank", "sel1", "sel0", "sel_counts"):
            assert np.array_equal(np.asarray(got[k]), np.asarray(want[k])), (rid, k)
    for rid in srv.resident_ids()[:4]:
        want = oracle_mod.build_all(host[rid], reqs[rid].sigma)
        got = srv.tree(rid).to_numpy()
        for k in ("bits", "C", "rank", "sel1", "sel0", "sel_counts"):
            assert np.array_equal(np.asarray(got[k], np.uint64).reshape(-1), np.asarray(want[k], np.uint64).reshape(-1))
    # Query answers: naive counting over the inputs.
    assert srv.results, "no query batch ran"
    for qid, out in srv.results.items():
        qb = issued[qid]
        tree = qb.tree.cpu().numpy()
        kind = qb.kind.cpu().numpy()
        a = qb.a.cpu().numpy()
        b = qb.b.cpu().numpy()
        got = out.cpu().numpy()
        for q in range(0, tree.size, 7):
            S = host[qb.targets[tree[q]]]
            if kind[q] == wt.Q_ACCESS:
                want = int(S[a[q]])
            elif kind[q] == wt.Q_RANK:
                want = int(np.count_nonzero(S[:b[q]] == a[q]))
            else:
                pos = np.flatnonzero(S == a[q])
                want = int(pos[b[q] - 1]) if 1 <= b[q] <= pos.size else -1
            assert got[q] == want, (qid, q, int(kind[q]), int(a[q]), int(b[q]), int(got[q]), want)


def test_serving_budget_holds_under_eviction(mods):
    """Device memory held by the server (resident trees, batch slabs, builds
    in flight) stays within its budget while it evicts: a batch slab stays
    charged whole until its last tree is evicted."""
    wt, serve = mods
    reqs, qtimes = inputs.serving_arrivals(0.08, rate=2000.0, qrate=100.0, n_exp=(10.0, 18.0),
                                           sigma_exp=(2.0, 16.0), index=11, max_requests=150)
    slab, layout, views = inputs.stage_requests(reqs)
    torch.cuda.synchronize()
    outputs = sum(serve.Server.footprint(r.n, r.sigma, layout[i][1])[0] for i, r in enumerate(reqs))
    budget = outputs // 4  # a quarter of the trees fit: the server must evict
    srv = serve.Server(budget_bytes=budget, small_n=1 << 15, small_sigma=1 << 12)
    torch.cuda.empty_cache()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    stats = serve.run_trace(srv, reqs, views, qtimes, slab, layout, qsize=2000, seed=5)
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() - base
    print(f"[serve] budget {budget >> 20} MiB, peak {peak >> 20} MiB, evictions {stats.evictions}, "
          f"batches {stats.batches}", flush=True)
    assert stats.failed == [] and stats.evictions > 0 and stats.batches > 0
    assert srv.in_use <= budget
    assert peak <= budget + (8 << 20), (peak, budget)
