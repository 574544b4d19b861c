"""Serving on the GPU: continuous batching over two streams; every query's
result in the mix equals its result alone and the oracle's; a query past its
budget is stopped without stopping the rest of its batch."""
import numpy as np
import pytest

from paper_2502_00317_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    from paper_2502_00317_amd import dist
    dist.lib()
    return dist


@pytest.mark.parametrize("pivot_k", [0, 5])
def test_served_equals_alone(D, oracle_mod, pivot_k):
    """Every served result equals the same query alone and the oracle: two
    lanes, and one bulk lane whose pool queries of k >= 5 take the pivot
    path."""
    from paper_2502_00317_amd.serve import DeviceBackend, Query, Server, oriented_bytes, replay, summarize
    pool = [gg.chung_lu(int(n), 2.4, 12.0, None, [31, i], plants=[10, 12])
            for i, n in enumerate(np.geomspace(2000, 20000, 6))]
    be = DeviceBackend(slots=2, grid_pcts=[40, 60], slot_cfgs=[{"budget_from_pair_start": 1}, {}])
    handles = {i: D.orient(g.row_ptr, g.col) for i, g in enumerate(pool)}
    pool_bytes = sum(oriented_bytes(g.n, g.m) for g in pool)
    rng = np.random.default_rng(5)
    t = np.cumsum(rng.exponential(1 / 500.0, size=150))
    qs = []
    for i in range(150):
        k = int(rng.integers(3, 9))
        if rng.random() < 0.1:
            a = gg.chung_lu(int(rng.integers(500, 3000)), 2.5, 10.0, None, [32, i], plants=[9])
            qs.append(Query(qid=i, k=k, t_arrival=float(t[i]), adhoc=(a.row_ptr, a.col), deadline_ms=30000))
        else:
            qs.append(Query(qid=i, k=k, t_arrival=float(t[i]), graph=int(rng.integers(0, len(pool))),
                            deadline_ms=30000))
    srv = Server(be, handles, slots=2, pool_bytes=pool_bytes, mem_limit=pool_bytes + (64 << 20),
                 express_ms=0 if pivot_k else 5, pivot_k=pivot_k)
    srv.start()
    replay(srv, qs)
    srv.stop()
    s = summarize(qs, max(q.t_done for q in qs))
    print(s, flush=True)
    assert s["completed"] == len(qs), [q.status for q in qs if q.status != "ok"]
    assert len(srv.batches) < len(qs)  # queries were batched
    print("moved to the bulk lane:", srv.demoted, "pivot passes:", srv.pivot_passes, flush=True)
    if pivot_k:
        assert srv.pivot_passes >= 1  # without an express lane every pool query of k >= 5 takes the path
    P61 = (1 << 61) - 1
    oracle_of = {}

    def pool_oracle(gi, k):
        # k <= 6 by enumeration, larger k by the pivot-based counter over
        # every root (pinned against enumeration); both are the oracle's
        if (gi, k) not in oracle_of:
            g = pool[gi]
            if k <= 6:
                oracle_of[gi, k] = oracle_mod.count(g.row_ptr, g.col, k)
            else:
                per = oracle_mod.pivot_count_roots(g.row_ptr, g.col, k, np.arange(g.n, dtype=np.int32))
                oracle_of[gi, k] = (sum(c for c, _ in per), sum(f for _, f in per) % P61)
        return oracle_of[gi, k]

    for q in qs:
        if q.adhoc is not None:
            G = D.orient(q.adhoc[0], q.adhoc[1])
            alone = D.count(G, q.k)[:2]
            want = oracle_mod.count(q.adhoc[0], q.adhoc[1], q.k)
            G.free()
        else:
            alone = D.count(handles[q.graph], q.k)[:2]
            want = pool_oracle(q.graph, q.k)
        assert (q.count, q.fp) == alone == want, q.qid


def test_pair_budget_stops_only_that_pair(D, oracle_mod):
    heavy = gg.gnp(300, 0.9, 3)       # about 1e13 20-cliques: far beyond the budget
    light = gg.small_powerlaw()
    Gh = D.orient(heavy.row_ptr, heavy.col)
    Gl = D.orient(light.row_ptr, light.col)
    res, rc, ms, st = D.count_batch([Gh, Gl, Gl], [20, 4, 5], use_graph=False,
                                    deadlines_ms=[300, 300, 300], with_status=True)
    assert st[0] == D.E_CANCELLED
    assert st[1] == D.OK and st[2] == D.OK
    assert res[1] == oracle_mod.count(light.row_ptr, light.col, 4)
    assert res[2] == oracle_mod.count(light.row_ptr, light.col, 5)
    assert ms < 5000


def test_stream_budget_and_early_reports(D, oracle_mod):
    """Streaming: light pairs are reported before the heavy pair is stopped
    by its budget; the heavy pair is reported as cancelled."""
    import time
    heavy = gg.gnp(300, 0.9, 3)
    light = gg.small_powerlaw()
    Gh = D.orient(heavy.row_ptr, heavy.col)
    Gl = D.orient(light.row_ptr, light.col)
    t0 = time.perf_counter()
    when = {}

    def on_done(i, c, f, st, dms):
        when[i] = (time.perf_counter() - t0, st)

    res, rc, st = D.count_batch_stream([Gh, Gl, Gl], [20, 4, 5], on_done,
                                       deadlines_ms=[400, 400, 400])
    assert st == [D.E_CANCELLED, D.OK, D.OK]
    assert res[1] == oracle_mod.count(light.row_ptr, light.col, 4)
    assert res[2] == oracle_mod.count(light.row_ptr, light.col, 5)
    assert when[0][1] == D.E_CANCELLED and when[1][1] == D.OK
    assert when[1][0] < when[0][0] and when[2][0] < when[0][0]


def test_budget_origin_pair_or_batch(D, oracle_mod):
    """budget_from_pair_start: with the heavy pair scheduled first, light
    pairs still get their whole budget when it runs from their own start,
    and none of it when it runs from the batch start."""
    heavy = gg.gnp(300, 0.9, 3)
    light = gg.small_powerlaw()
    Gh = D.orient(heavy.row_ptr, heavy.col)
    Gl = D.orient(light.row_ptr, light.col)
    want4 = oracle_mod.count(light.row_ptr, light.col, 4)
    want5 = oracle_mod.count(light.row_ptr, light.col, 5)
    got = {}

    def on_done(i, c, f, st, dms):
        got[i] = (st, dms)

    cfg = D.config(budget_from_pair_start=1)
    res, rc, st = D.count_batch_stream([Gh, Gl, Gl], [20, 4, 5], on_done, cfg=cfg,
                                       deadlines_ms=[300, 300, 300], costs=[1.0, 1e6, 1e6])
    assert st == [D.E_CANCELLED, D.OK, D.OK]
    assert res[1] == want4 and res[2] == want5
    assert 250 <= got[0][1] < 5000          # the heavy pair ran about its budget
    assert 0 <= got[1][1] < 300 and 0 <= got[2][1] < 300
    res, rc, st = D.count_batch_stream([Gh, Gl, Gl], [20, 4, 5], on_done, cfg=D.config(),
                                       deadlines_ms=[300, 300, 300], costs=[1.0, 1e6, 1e6])
    assert st == [D.E_CANCELLED, D.E_CANCELLED, D.E_CANCELLED]
