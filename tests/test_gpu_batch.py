"""Batched counting (dist_count_batch): every pair's result equals the
oracle's and the plain per-graph call's; graph replays repeat the eager
result; width merging leaves results unchanged."""
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


def _small_batch(seed=11, count=40):
    rng = np.random.default_rng(seed)
    graphs, ks = [], []
    for i in range(count):
        n = int(rng.integers(20, 600))
        plants = [int(x) for x in rng.integers(6, 16, size=int(rng.integers(0, 3)))]
        g = gg.chung_lu(n, float(rng.uniform(2.1, 3.0)), float(min(rng.uniform(4, 20), (n - 1) / 2)),
                        None, [seed, i], plants=plants)
        graphs.append(g)
        ks.append(int(rng.integers(1, 10)))
    graphs.append(gg.empty(5)); ks.append(3)
    graphs.append(gg.complete(90)); ks.append(6)
    graphs.append(gg.turan(100, 9)); ks.append(7)
    return graphs, ks


def test_batch_matches_oracle(D, oracle_mod):
    graphs, ks = _small_batch()
    G = [D.orient(g.row_ptr, g.col, order=D.ORDER_DEGENERACY if i % 2 else D.ORDER_DEGREE)
         for i, g in enumerate(graphs)]
    want = [oracle_mod.count(g.row_ptr, g.col, k) for g, k in zip(graphs, ks)]
    for cfg, use_graph in ((D.config(), True), (D.config(), False), (D.config(memo=0), True),
                           (D.config(min_width=4), True), (D.config(memo=2, prune=0), False)):
        got, rc, ms = D.count_batch(G, ks, cfg=cfg, use_graph=use_graph)
        assert rc in (D.OK, D.E_OVERFLOW)
        assert got == want


def test_batch_same_graph_many_k(D, oracle_mod):
    g = gg.small_powerlaw()
    G = D.orient(g.row_ptr, g.col)
    ks = [1, 2, 3, 4, 5, 6, 3, 4]
    got, rc, _ = D.count_batch([G] * len(ks), ks)
    assert got == [oracle_mod.count(g.row_ptr, g.col, k) for k in ks]


def test_graph_replays_repeat_eager(D):
    """The captured launch sequence is replayed several times with eager
    work and synchronisations in between; every replay equals the eager
    per-graph results (memo tags are renewed per replay)."""
    import torch
    graphs, ks = _small_batch(seed=12, count=30)
    G = [D.orient(g.row_ptr, g.col) for g in graphs]
    eager = [D.count(Gi, k)[:2] for Gi, k in zip(G, ks)]
    for rep in range(4):
        got, rc, _ = D.count_batch(G, ks, use_graph=True)
        assert got == eager, rep
        # eager work between replays
        D.count(G[rep], ks[rep])
        torch.cuda.synchronize()


def test_stream_reports_every_pair_once(D, oracle_mod):
    """dist_count_batch_stream: each pair is reported exactly once, with the
    same result the batch returns and the oracle computes; graphs of every
    width class, k = 1 and pairs with no deep-enough root included."""
    import threading
    graphs, ks = _small_batch(seed=13, count=40)
    G = [D.orient(g.row_ptr, g.col) for g in graphs]
    want = [oracle_mod.count(g.row_ptr, g.col, k) for g, k in zip(graphs, ks)]
    seen = {}
    me = threading.get_ident()

    def on_done(i, c, f, st, dms):
        assert threading.get_ident() == me
        assert i not in seen
        seen[i] = ((c, f), st)

    for cfg in (D.config(), D.config(grid_pct=25, fingerprint=1), D.config(memo=0, chunk_work=64)):
        seen.clear()
        res, rc, st = D.count_batch_stream(G, ks, on_done, cfg=cfg)
        assert rc in (D.OK, D.E_OVERFLOW)
        assert res == want
        assert sorted(seen) == list(range(len(G)))
        for i in range(len(G)):
            assert seen[i] == (want[i], st[i]), i


def test_estimate_cost_orders_work(D):
    g = gg.complete(40)
    G = D.orient(g.row_ptr, g.col)
    import math
    # complete graph: out-degrees 0..39, cost = sum_d C(d, k-1) = C(40, k)
    for k in (2, 3, 5, 8):
        assert abs(D.estimate_cost(G, k) - math.comb(40, k)) <= 1e-9 * math.comb(40, k) + 1e-6
    z = gg.empty(4)
    e = D.orient(z.row_ptr, z.col)
    assert D.estimate_cost(e, 3) == 0.0


def test_per_pair_switches(D, oracle_mod):
    """dist_count_batch_tuned: random per-pair (min_width, chunk_work, memo)
    give every pair the oracle's result, in replays of the captured graph
    too; new switches are planned afresh; a switch out of range is
    rejected."""
    graphs, ks = _small_batch(seed=23)
    G = [D.orient(g.row_ptr, g.col) for g in graphs]
    want = [oracle_mod.count(g.row_ptr, g.col, k) for g, k in zip(graphs, ks)]
    rng = np.random.default_rng(5)
    for trial in range(3):
        sw = [dict(min_width=int(rng.choice([0, 1, 2, 4, 8])), chunk_work=int(rng.choice([-1, 0, 64, 512])),
                   memo=int(rng.choice([-1, 0, 1, 2]))) for _ in ks]
        for rep in range(3):
            print("tuned batch", trial, rep, flush=True)
            got, rc, ms = D.count_batch_tuned(G, ks, sw, cfg=D.config(memo=1), use_graph=True)
            assert rc in (D.OK, D.E_OVERFLOW)
            assert got == want, (trial, rep)
    with pytest.raises(D.DistError):
        D.count_batch_tuned(G, ks, [dict(memo=3)] * len(ks))


def test_per_bucket_autotune(D, oracle_mod, tmp_path):
    """The per-bucket autotuner: buckets by (width class, k band), two
    candidates timed per bucket, winners stored in its database and reused
    on a second call; the batch run with the per-pair winners equals the
    oracle."""
    from paper_2502_00317_amd import autotune
    graphs, ks = _small_batch(seed=31)
    G = [D.orient(g.row_ptr, g.col) for g in graphs]
    want = [oracle_mod.count(g.row_ptr, g.col, k) for g, k in zip(graphs, ks)]
    cands = [dict(min_width=1, chunk_work=512, memo=1), dict(min_width=2, chunk_work=0, memo=0)]
    db = autotune.TuningDB(str(tmp_path / "db.json"))
    per_pair, buckets = autotune.tune_buckets(D, G, ks, db=db, candidates=cands, reps=1)
    assert sum(e["pairs"] for e in buckets.values()) == len(ks)
    assert all(e["switches"] in cands for e in buckets.values())
    got, rc, _ = D.count_batch_tuned(G, ks, per_pair, use_graph=True)
    assert got == want
    again, _ = autotune.tune_buckets(D, G, ks, db=autotune.TuningDB(str(tmp_path / "db.json")), candidates=cands)
    assert again == per_pair
