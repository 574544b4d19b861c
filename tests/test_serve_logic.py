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


def test_streamed_completion_cheap_first(oracle_mod):
    """A cheap query batched with an expensive one completes when its own
    result is known, not when the batch ends; results stay exact."""
    graphs, handles = _pool(2)
    cost = lambda g, k: 200.0 if k == 6 else 1.0
    be = FakeBackend(oracle_mod, cost, seconds_per_cost=1e-3)
    srv = Server(be, handles, slots=1)
    qs = [Query(qid=0, k=6, t_arrival=0.0, graph=1),
          Query(qid=1, k=3, t_arrival=0.0, graph=0),
          Query(qid=2, k=4, t_arrival=0.0, graph=0)]
    srv.start()
    replay(srv, qs)
    srv.stop()
    assert all(q.status == "ok" for q in qs)
    for q in qs:
        g = graphs[q.graph]
        assert (q.count, q.fp) == oracle_mod.count(g.row_ptr, g.col, q.k)
    if len(be.calls) == 1:  # all three went into one batch
        assert qs[1].t_done < qs[0].t_done - 0.1 and qs[2].t_done < qs[0].t_done - 0.1
    # without streaming every query of a batch ends with the batch
    srv2 = Server(FakeBackend(oracle_mod, cost, seconds_per_cost=1e-3), handles, slots=1,
                  stream_results=False)
    qs2 = [Query(qid=q.qid, k=q.k, t_arrival=0.0, graph=q.graph) for q in qs]
    srv2.start()
    replay(srv2, qs2)
    srv2.stop()
    if len(srv2.batches) == 1:
        assert len({q.t_done for q in qs2}) == 1


def test_express_lane_moves_heavy_queries(oracle_mod):
    """Slot 0 is an express lane with a 20 ms device budget.  A heavy query
    cut off there moves to the bulk lane and still completes exactly; a later
    query with the same (graph, k) goes to the bulk lane directly; light
    queries are not held behind heavy ones."""
    graphs, handles = _pool(3)
    cost = lambda g, k: 150.0 if k == 6 else 1.0      # 150 ms vs 1 ms
    be = FakeBackend(oracle_mod, cost, seconds_per_cost=1e-3)
    srv = Server(be, handles, slots=2, express_ms=20)
    qs = [Query(qid=0, k=6, t_arrival=0.0, graph=1, deadline_ms=5000)]
    qs += [Query(qid=1 + i, k=3 + i % 3, t_arrival=0.01 * i, graph=i % 3, deadline_ms=5000) for i in range(20)]
    qs += [Query(qid=50, k=6, t_arrival=0.5, graph=1, deadline_ms=5000)]
    srv.start()
    replay(srv, qs)
    srv.stop()
    for q in qs:
        assert q.status == "ok", (q.qid, q.status)
        g = graphs[q.graph]
        assert (q.count, q.fp) == oracle_mod.count(g.row_ptr, g.col, q.k)
    assert qs[0].moves == 1 and qs[0].lane == "bulk"
    assert qs[-1].moves == 0 and qs[-1].lane == "bulk"     # known heavy: bulk lane directly
    assert (1, 6) in srv.heavy and srv.demoted == 1
    light = [q.latency for q in qs[1:-1]]
    assert max(light) < 0.12, light                          # never waited for the 150 ms query


def test_express_moves_keep_adhoc_memory_once(oracle_mod):
    graphs, handles = _pool(1)
    pool_bytes = sum(h.nbytes for h in handles.values())
    a = gg.chung_lu(800, 2.5, 8.0, None, [21, 0])
    cost = lambda g, k: 100.0 if g.n == a.n else 1.0
    be = FakeBackend(oracle_mod, cost, seconds_per_cost=1e-3, pool_bytes=pool_bytes)
    srv = Server(be, handles, slots=3, express_ms=10, pool_bytes=pool_bytes)
    qs = [Query(qid=0, k=4, t_arrival=0.0, adhoc=(a.row_ptr, a.col), deadline_ms=5000),
          Query(qid=1, k=3, t_arrival=0.0, graph=0, deadline_ms=5000)]
    srv.start()
    replay(srv, qs)
    srv.stop()
    assert [q.status for q in qs] == ["ok", "ok"]
    assert qs[0].moves == 1
    assert (qs[0].count, qs[0].fp) == oracle_mod.count(a.row_ptr, a.col, 4)
    assert srv.mem_used == pool_bytes and be.live == pool_bytes   # oriented once, freed once


def test_plain_mode_one_query_at_a_time(oracle_mod):
    graphs, handles = _pool(2)
    be = FakeBackend(oracle_mod, _cost, seconds_per_cost=1e-3)
    srv = Server(be, handles, slots=1, plain=True)
    qs = [Query(qid=i, k=3 + i % 4, t_arrival=0.0, graph=i % 2) for i in range(8)]
    srv.start()
    replay(srv, qs)
    srv.stop()
    assert all(b[1] == 1 for b in srv.batches) and len(srv.batches) == 8
    for q in qs:
        g = graphs[q.graph]
        assert (q.count, q.fp) == oracle_mod.count(g.row_ptr, g.col, q.k)


def test_budget_spent_in_queue_is_dnf(oracle_mod):
    graphs, handles = _pool(1)
    be = FakeBackend(oracle_mod, lambda g, k: 300.0, seconds_per_cost=1e-3)
    srv = Server(be, handles, slots=1, max_batch=1)
    qs = [Query(qid=0, k=3, t_arrival=0.0, graph=0, deadline_ms=1000),
          Query(qid=1, k=4, t_arrival=0.0, graph=0, deadline_ms=100)]
    srv.start()
    replay(srv, qs)
    srv.stop()
    assert qs[0].status == "ok" and qs[1].status == "dnf"


def test_route_by_learned_threshold(oracle_mod):
    """Once a query with estimate E was cut off in the express lane, a new
    (graph, k) with an estimate above E goes to the bulk lane on arrival;
    one below the largest completed estimate stays in the express lane."""
    graphs, handles = _pool(4)              # n = 200, 350, 500, 650
    cost = lambda g, k: 120.0 if g.n >= 500 else 1.0
    be = FakeBackend(oracle_mod, cost, seconds_per_cost=1e-3, estimate_fn=lambda g, k: float(g.n))
    srv = Server(be, handles, slots=2, express_ms=20)
    srv.start()
    first = [Query(qid=0, k=4, t_arrival=0.0, graph=2, deadline_ms=5000),
             Query(qid=1, k=4, t_arrival=0.0, graph=0, deadline_ms=5000)]
    replay(srv, first)
    assert first[0].moves == 1 and first[1].lane == "express"
    assert srv.heavy_min[4] == 500.0 and srv.light_max[4] == 200.0
    t = srv.now()
    second = [Query(qid=2, k=4, t_arrival=t, graph=3, deadline_ms=5000),   # 650 >= 500: bulk
              Query(qid=3, k=4, t_arrival=t, graph=1, deadline_ms=5000),   # 350: express
              Query(qid=4, k=5, t_arrival=t, graph=3, deadline_ms=5000)]   # k = 5 not learned yet
    replay(srv, second)
    srv.stop()
    assert second[0].lane == "bulk" and second[0].moves == 0
    assert second[1].lane == "express"
    assert second[2].moves == 1
    assert srv.routed_bulk == 1
    for q in first + second:
        assert q.status == "ok"
        g = graphs[q.graph]
        assert (q.count, q.fp) == oracle_mod.count(g.row_ptr, g.col, q.k)


def test_express_batches_bounded_by_predicted_time(oracle_mod):
    """An express batch takes never-seen queries only while their predicted
    time (express_ms each) fits express_batch_ms."""
    graphs, handles = _pool(3)
    be = FakeBackend(oracle_mod, lambda g, k: 2.0, seconds_per_cost=1e-3)
    srv = Server(be, handles, slots=2, express_ms=10, express_batch_ms=30)
    qs = [Query(qid=i, k=3 + i % 5, t_arrival=0.0, graph=i % 3, deadline_ms=10000) for i in range(12)]
    srv.start()
    replay(srv, qs)
    srv.stop()
    assert all(q.status == "ok" for q in qs)
    express = [b for b in srv.batches if b[0] == 0 and b[1] > 0]
    assert max(b[1] for b in express) <= 3


def test_shed_queries_known_to_exceed_budget(oracle_mod):
    """A (graph, k) cut off in the bulk lane after running for at least
    shed_frac of the budget is reported DNF at once when it comes again."""
    graphs, handles = _pool(2)
    cost = lambda g, k: 10000.0 if k == 8 else 1.0
    be = FakeBackend(oracle_mod, cost, seconds_per_cost=1e-3)
    srv = Server(be, handles, slots=2, express_ms=10, shed_frac=0.5)
    srv.start()
    first = [Query(qid=0, k=8, t_arrival=0.0, graph=1, deadline_ms=300)]
    replay(srv, first)
    t = srv.now()
    second = [Query(qid=1, k=8, t_arrival=t, graph=1, deadline_ms=300),
              Query(qid=2, k=3, t_arrival=t, graph=1, deadline_ms=300)]
    replay(srv, second)
    srv.stop()
    assert first[0].status == "dnf" and first[0].moves == 1
    assert second[0].status == "dnf" and second[0].lane == "shed" and srv.shed == 1
    assert second[0].latency < 0.05
    assert second[1].status == "ok"


def test_summary_charges_unfinished_queries_their_budget():
    """Percentiles count every query: a DNF or shed query at its latency
    budget, so dropping work cannot improve p50/p99; the completed-only
    figures are reported beside them."""
    qs = []
    for i in range(100):
        q = Query(qid=i, k=4, t_arrival=0.0, graph=0, deadline_ms=2000)
        if i < 90:
            q.status, q.t_done, q.count = "ok", 0.010, 1
        else:
            q.status = "dnf"
            if i >= 95:
                q.lane = "shed"
        qs.append(q)
    s = summarize(qs, 1.0)
    assert s["completed"] == 90 and s["dnf"] == 10 and s["shed"] == 5
    assert s["dnf_rate"] == 0.1
    assert abs(s["p50_ms"] - 10.0) < 1e-6
    assert abs(s["p99_ms"] - 2000.0) < 1e-6          # the unfinished tail, at its budget
    assert abs(s["p99_completed_ms"] - 10.0) < 1e-6


def test_router_table_round_trip_and_frozen_routing(oracle_mod):
    """The routing state learned in one run, stored and loaded into a new
    server with learning off, routes a new query by the stored threshold
    (no express attempt), and stays unchanged by the run."""
    import json
    graphs, handles = _pool(4)              # n = 200, 350, 500, 650
    cost = lambda g, k: 120.0 if g.n >= 500 else 1.0
    mk = lambda: FakeBackend(oracle_mod, cost, seconds_per_cost=1e-3, estimate_fn=lambda g, k: float(g.n))
    srv = Server(mk(), handles, slots=2, express_ms=20)
    srv.start()
    replay(srv, [Query(qid=0, k=4, t_arrival=0.0, graph=2, deadline_ms=5000),
                 Query(qid=1, k=4, t_arrival=0.0, graph=0, deadline_ms=5000)])
    srv.stop()
    table = json.loads(json.dumps(srv.router_state()))   # as stored on disk
    assert table["heavy_min"] == {"4": 500.0} and table["light_max"] == {"4": 200.0}
    assert table["heavy"] == [[2, 4]]
    frozen = Server(mk(), handles, slots=2, express_ms=20, router_table=table, learn=False)
    assert frozen.router_state() == table
    frozen.start()
    qs = [Query(qid=2, k=4, t_arrival=0.0, graph=3, deadline_ms=5000),   # 650 >= 500: bulk at once
          Query(qid=3, k=4, t_arrival=0.0, graph=1, deadline_ms=5000),   # 350: express
          Query(qid=4, k=5, t_arrival=0.0, graph=3, deadline_ms=5000)]   # k = 5: express, cut, bulk
    replay(frozen, qs)
    frozen.stop()
    assert qs[0].lane == "bulk" and qs[0].moves == 0
    assert qs[1].lane == "express"
    assert qs[2].moves == 1
    assert frozen.router_state() == table                                # nothing learned
    for q in qs:
        g = graphs[q.graph]
        assert q.status == "ok" and (q.count, q.fp) == oracle_mod.count(g.row_ptr, g.col, q.k)


def test_frozen_router_repeats_lanes(oracle_mod):
    """Two runs of one seeded stream under the same frozen table take the
    same lane decisions for every query."""
    graphs, handles = _pool(4)
    cost = lambda g, k: 60.0 if (g.n >= 500 and k >= 5) else 1.0
    table = {"heavy_min": {"5": 500.0}, "light_max": {"5": 350.0}, "heavy": [[3, 6]]}
    runs = []
    for _ in range(2):
        be = FakeBackend(oracle_mod, cost, seconds_per_cost=1e-3, estimate_fn=lambda g, k: float(g.n))
        srv = Server(be, handles, slots=2, express_ms=20, router_table=table, learn=False)
        rng = np.random.default_rng(11)
        t = np.cumsum(rng.exponential(1 / 200.0, size=40))
        qs = [Query(qid=i, k=int(rng.integers(3, 7)), t_arrival=float(t[i]), graph=int(rng.integers(0, 4)),
                    deadline_ms=5000) for i in range(40)]
        srv.start()
        replay(srv, qs)
        srv.stop()
        assert all(q.status == "ok" for q in qs)
        runs.append([(q.lane, q.moves) for q in qs])
    assert runs[0] == runs[1]


def test_bulk_pivot_pass_answers_queued_k(oracle_mod):
    """With pivot_k, the bulk lane answers its pool queries of k >= pivot_k
    with one all-k pass per graph of what is queued: exact results, and
    sooner than the search would (120 ms per query here against 30 ms per
    pass)."""
    graphs, handles = _pool(2)
    cost = lambda g, k: 120.0 if k >= 6 else 1.0
    be = FakeBackend(oracle_mod, cost, seconds_per_cost=1e-3, pivot_cost_fn=lambda g, kmax: 30.0)
    srv = Server(be, handles, slots=2, express_ms=10, pivot_k=6)
    qs = [Query(qid=i, k=6 + i % 3, t_arrival=0.0, graph=i % 2, deadline_ms=5000) for i in range(6)]
    qs += [Query(qid=10 + i, k=3 + i % 2, t_arrival=0.0, graph=i % 2, deadline_ms=5000) for i in range(4)]
    srv.start()
    replay(srv, qs)
    srv.stop()
    for q in qs:
        g = graphs[q.graph]
        assert q.status == "ok" and (q.count, q.fp) == oracle_mod.count(g.row_ptr, g.col, q.k), q.qid
    # queries reach the bulk lane as the express lane cuts them off, so a pass
    # holds what is queued at the time: at most one pass per heavy query
    assert 1 <= srv.pivot_passes <= 6 and len(be.pivot_calls) == srv.pivot_passes
    assert max(q.latency for q in qs[:6]) < 0.5


def test_bulk_pivot_pass_too_slow_falls_back(oracle_mod):
    """A pivot pass that runs out of its budget marks the graph slow; its
    queries go back to the search, which completes them exactly, and the
    graph is not passed to pivoting again."""
    graphs, handles = _pool(1)
    cost = lambda g, k: 40.0 if k >= 6 else 1.0
    be = FakeBackend(oracle_mod, cost, seconds_per_cost=1e-3, pivot_cost_fn=lambda g, kmax: 100000.0)
    srv = Server(be, handles, slots=2, express_ms=10, pivot_k=6)
    srv.start()
    first = [Query(qid=0, k=6, t_arrival=0.0, graph=0, deadline_ms=600)]
    replay(srv, first)
    t = srv.now()
    second = [Query(qid=1, k=7, t_arrival=t, graph=0, deadline_ms=600)]
    replay(srv, second)
    srv.stop()
    assert 0 in srv.pivot_slow and len(be.pivot_calls) == 1
    g = graphs[0]
    for q in second:
        assert q.status == "ok" and (q.count, q.fp) == oracle_mod.count(g.row_ptr, g.col, q.k)


def test_bulk_pivot_pass_without_deadlines(oracle_mod):
    """Queries without a latency budget give their pivot pass no deadline
    (not a 1 ms one): the pass completes and nothing is marked slow."""
    graphs, handles = _pool(1)
    be = FakeBackend(oracle_mod, lambda g, k: 1.0, seconds_per_cost=1e-3, pivot_cost_fn=lambda g, kmax: 20.0)
    srv = Server(be, handles, slots=1, pivot_k=6)
    qs = [Query(qid=i, k=6 + i, t_arrival=0.0, graph=0) for i in range(3)]
    srv.start()
    replay(srv, qs)
    srv.stop()
    g = graphs[0]
    assert srv.pivot_passes >= 1 and not srv.pivot_slow
    for q in qs:
        assert q.status == "ok" and (q.count, q.fp) == oracle_mod.count(g.row_ptr, g.col, q.k)
