"""Serving logic on a simulated device (CPU only): continuous batching over
several slots, memory-gated admission of ad-hoc graphs, per-query deadlines
and exact results."""
import threading

import numpy as np
import pytest

from paper_2502_00317_amd import graphgen as gg
from paper_2502_00317_amd.serve import Query, Server, oriented_bytes, replay, summarize
from fake_device import FakeBackend, FakeGraph


def _pool(n_graphs=4, seed=0):
    graphs = [gg.chung_lu(int(200 + 150 * i), 2.4, 8.0, None, [seed, i], plants=[8]) for i in range(n_graphs)]
    handles = {i: FakeGraph(g.row_ptr, g.col, oriented_bytes(g.n, g.m)) for i, g in enumerate(graphs)}
    return graphs, handles


def _cost(g, k):
    return 1.0 + 0.01 * g.n


def test_results_exact_and_slots_overlap(oracle_mod):
    graphs, handles = _pool()
    be = FakeBackend(oracle_mod, _cost, seconds_per_cost=2e-3)
    srv = Server(be, handles, slots=3)
    rng = np.random.default_rng(1)
    t = np.cumsum(rng.exponential(1 / 400.0, size=120))
    qs = [Query(qid=i, k=int(rng.integers(3, 7)), t_arrival=float(t[i]), graph=int(rng.integers(0, 4)))
          for i in range(120)]
    srv.start()
    replay(srv, qs)
    srv.stop()
    for q in qs:
        assert q.status == "ok"
        g = graphs[q.graph]
        assert (q.count, q.fp) == oracle_mod.count(g.row_ptr, g.col, q.k)
        assert q.latency >= 0
    # queries were batched (fewer calls than queries) and slots overlapped
    assert len(be.calls) < len(qs)
    assert be.max_active >= 2
    s = summarize(qs, 1.0)
    assert s["completed"] == 120 and s["dnf"] == 0


def test_memory_gating_never_overcommits(oracle_mod):
    graphs, handles = _pool(2)
    pool_bytes = sum(h.nbytes for h in handles.values())
    adhoc = [gg.chung_lu(3000, 2.5, 10.0, None, [7, i]) for i in range(6)]
    need = oriented_bytes(adhoc[0].n, adhoc[0].m)
    limit = pool_bytes + int(1.5 * max(oriented_bytes(a.n, a.m) for a in adhoc))  # one ad-hoc graph at a time
    be = FakeBackend(oracle_mod, _cost, seconds_per_cost=5e-4, pool_bytes=pool_bytes, mem_limit=limit)
    srv = Server(be, handles, slots=3, mem_limit=limit, pool_bytes=pool_bytes)
    qs = [Query(qid=i, k=3, t_arrival=0.0, adhoc=(a.row_ptr, a.col)) for i, a in enumerate(adhoc)]
    qs += [Query(qid=100 + i, k=4, t_arrival=0.0, graph=i % 2) for i in range(6)]
    srv.start()
    replay(srv, qs)
    srv.stop()
    assert all(q.status == "ok" for q in qs)
    assert srv.peak_mem <= limit and be.peak <= limit
    for q in qs[:6]:
        assert (q.count, q.fp) == oracle_mod.count(q.adhoc[0], q.adhoc[1], 3)
    # pool queries are not held behind ad-hoc ones waiting for memory
    last_pool = max(q.t_done for q in qs[6:])
    last_adhoc = max(q.t_done for q in qs[:6])
    assert last_pool <= last_adhoc
    assert srv.mem_used == pool_bytes


def test_oversized_upload_rejected(oracle_mod):
    graphs, handles = _pool(1)
    big = gg.chung_lu(5000, 2.5, 20.0, None, 9)
    srv = Server(FakeBackend(oracle_mod, _cost), handles, slots=1, mem_limit=1 << 20, pool_bytes=0)
    q = Query(qid=0, k=3, t_arrival=0.0, adhoc=(big.row_ptr, big.col))
    ok = Query(qid=1, k=3, t_arrival=0.0, graph=0)
    srv.start()
    replay(srv, [q, ok])
    srv.stop()
    assert q.status == "rejected" and ok.status == "ok"


def test_deadline_dnf_does_not_stop_the_batch(oracle_mod):
    graphs, handles = _pool(2)
    slow = lambda g, k: 1000.0 if k == 9 else 1.0
    be = FakeBackend(oracle_mod, slow, seconds_per_cost=1e-3)
    srv = Server(be, handles, slots=1)
    qs = [Query(qid=0, k=9, t_arrival=0.0, graph=1, deadline_ms=50),
          Query(qid=1, k=3, t_arrival=0.0, graph=0, deadline_ms=50),
          Query(qid=2, k=4, t_arrival=0.0, graph=1, deadline_ms=50)]
    srv.start()
    replay(srv, qs)
    srv.stop()
    assert [q.status for q in qs] == ["dnf", "ok", "ok"]
    s = summarize(qs, 1.0)
    assert s["dnf"] == 1 and s["completed"] == 2
