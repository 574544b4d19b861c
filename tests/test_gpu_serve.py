"""Serving on the GPU: continuous batching over two streams; every query's
result in the mix equals its result alone; a query past its budget is
stopped without stopping the rest of its batch."""
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


def test_served_equals_alone(D, oracle_mod):
    from paper_2502_00317_amd.serve import DeviceBackend, Query, Server, oriented_bytes, replay, summarize
    pool = [gg.chung_lu(int(n), 2.4, 12.0, None, [31, i], plants=[10, 12])
            for i, n in enumerate(np.geomspace(2000, 20000, 6))]
    be = DeviceBackend(slots=2)
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
    srv = Server(be, handles, slots=2, pool_bytes=pool_bytes, mem_limit=pool_bytes + (64 << 20))
    srv.start()
    replay(srv, qs)
    srv.stop()
    s = summarize(qs, max(q.t_done for q in qs))
    print(s, flush=True)
    assert s["completed"] == len(qs), [q.status for q in qs if q.status != "ok"]
    assert len(srv.batches) < len(qs)  # queries were batched
    for q in qs:
        if q.adhoc is not None:
            G = D.orient(q.adhoc[0], q.adhoc[1])
            alone = D.count(G, q.k)[:2]
            want = oracle_mod.count(q.adhoc[0], q.adhoc[1], q.k)
            G.free()
        else:
            alone = D.count(handles[q.graph], q.k)[:2]
            g = pool[q.graph]
            want = oracle_mod.count(g.row_ptr, g.col, q.k) if q.k <= 6 else alone
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
