"""dist_list through the C ABI: every clique exactly once, each row sorted,
the same set as the oracle's listing (CPU reference) and the same count
and fingerprint as dist_count."""
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


def _sorted_rows(a):
    a = np.asarray(a)
    if len(a) == 0:
        return a
    return a[np.lexsort(a.T[::-1])]


def _check(D, oracle_mod, g, k, order):
    G = D.orient(g.row_ptr, g.col, order=order)
    rows, cnt, fp, rc = D.list_cliques(G, k)
    assert rc in (D.OK, D.E_OVERFLOW)
    want = oracle_mod.list_cliques(g.row_ptr, g.col, k)
    assert rows.shape == want.shape, (rows.shape, want.shape)
    if len(rows):
        assert np.all(rows[:, 1:] > rows[:, :-1]), "rows not strictly ascending"
    assert np.array_equal(_sorted_rows(rows), want)
    assert (cnt, fp) == oracle_mod.count(g.row_ptr, g.col, k)


def test_fig2_list(D, oracle_mod):
    g = gg.fig2()
    for order in (D.ORDER_DEGREE, D.ORDER_DEGENERACY, D.ORDER_INPUT):
        for k in range(1, 8):
            print("fig2 list", order, k, flush=True)
            _check(D, oracle_mod, g, k, order)


@pytest.mark.parametrize("seed", range(6))
def test_random_list(D, oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 90))
    g = gg.gnp(n, float(rng.uniform(0.2, 0.8)), 700 + seed)
    for k in (2, 3, 4, 5, 6, 7):
        print("gnp list", seed, n, k, flush=True)
        _check(D, oracle_mod, g, k, D.ORDER_DEGREE)


def test_complete_and_turan_list(D, oracle_mod):
    for g, ks in ((gg.complete(70), (3, 4, 5)), (gg.turan(60, 8), (4, 5, 6)), (gg.complete(130), (3, 4))):
        for k in ks:
            print("list", g.name, k, flush=True)
            _check(D, oracle_mod, g, k, D.ORDER_DEGENERACY)


def test_small_powerlaw_list(D, oracle_mod):
    g = gg.small_powerlaw()
    for k in (3, 4, 5):
        print("cfg1 list", k, flush=True)
        _check(D, oracle_mod, g, k, D.ORDER_DEGREE)


def test_list_sink_cancel(D):
    g = gg.complete(40)
    G = D.orient(g.row_ptr, g.col)
    calls = []

    def sink(rows):
        calls.append(len(rows))
        return 1  # stop

    _, cnt, fp, rc = D.list_cliques(G, 4, sink=sink)
    assert rc == D.E_CANCELLED
    assert len(calls) == 1


LIST_CONFIGS = [dict(memo=1), dict(memo=2), dict(memo=0), dict(memo=2, prune=0), dict(memo=2, trie_nodes=8)]


def _check_cfg(D, oracle_mod, g, k, order, cfg):
    G = D.orient(g.row_ptr, g.col, order=order)
    rows, cnt, fp, rc = D.list_cliques(G, k, cfg=D.config(**cfg))
    assert rc in (D.OK, D.E_OVERFLOW)
    want = oracle_mod.list_cliques(g.row_ptr, g.col, k)
    assert rows.shape == want.shape, (rows.shape, want.shape, cfg)
    if len(rows):
        assert np.all(rows[:, 1:] > rows[:, :-1]), "rows not strictly ascending"
    assert np.array_equal(_sorted_rows(rows), want), cfg
    assert (cnt, fp) == oracle_mod.count(g.row_ptr, g.col, k), cfg
    return G.stats()


def test_trie_listing_switches(D, oracle_mod):
    """ListingDense on the Induced Subgraph Trie (criterion (1), or forced on
    every branch), plain Listing, no pruning, and a node pool of 8 (frames
    that cannot insert their string list without the trie): the same clique
    set as the oracle in every case; forced tries do retrieve."""
    cases = [(gg.fig2(), (3, 4, 5), D.ORDER_DEGENERACY), (gg.turan(40, 6), (4, 5, 6), D.ORDER_DEGREE),
             (gg.gnp(45, 0.6, 9), (4, 5, 6, 7), D.ORDER_DEGREE), (gg.complete(30), (4, 6), D.ORDER_DEGREE)]
    hits = 0
    for g, ks, order in cases:
        for k in ks:
            for cfg in LIST_CONFIGS:
                print("trie list", g.name, k, cfg, flush=True)
                st = _check_cfg(D, oracle_mod, g, k, order, cfg)
                if cfg.get("memo") == 2 and "trie_nodes" not in cfg:
                    assert st.memo_inserts > 0
                    hits += st.memo_hits
    assert hits > 0, "no l-memoised node was ever reused"


def test_trie_listing_powerlaw(D, oracle_mod):
    g = gg.small_powerlaw()
    for k in (4, 5, 6):
        for cfg in (dict(memo=1), dict(memo=2)):
            print("cfg1 trie list", k, cfg, flush=True)
            _check_cfg(D, oracle_mod, g, k, D.ORDER_DEGREE, cfg)


def _fig2_trie(D):
    import json
    import os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "fig2.json")))
    g = gg.fig2()
    # the worked example's order u0 < u1 < ... < u8 (a degeneracy order of
    # Figure 2), taken as given
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_INPUT)
    assert list(G.ranks()) == list(range(9))
    return fx, g, G


def test_example4_links_and_retrieval(D):
    """The paper's Example 4: for root u0 and k = 4, with ListingDense on
    every branch, the trie holds the prefixes of the identifying strings of
    Table 2 that u0's search inserts, the l-child and l-sibling links of
    t1 .. t6 are those printed, and ListingIST(t1, 3, {u0}) yields the three
    4-cliques containing u0."""
    fx, g, G = _fig2_trie(D)
    ex = fx["example4"]
    loc = None
    out = None
    # first call learns the local ids of u0's out-neighbours
    out = D.ist_inspect(G, 4, 0, cfg=D.config(memo=2))
    loc = [int(v) for v in out["local_ids"]]
    assert loc == fx["out_neighbours"]["0"]
    t1 = set(ex["nodes"]["t1"])
    bits = sum(1 << i for i, v in enumerate(loc) if v in t1)
    out = D.ist_inspect(G, 4, 0, cfg=D.config(memo=2), ret_set=[bits], ret_l=3)
    nodes = out["nodes"]
    idx = {s: i for i, s in enumerate(nodes)}
    assert len(idx) == len(nodes), "a vertex set has two nodes"
    want_sets = {frozenset(v) for v in ex["nodes"].values()} | {frozenset([7, 5, 4, 3])}
    assert set(nodes[1:]) == want_sets
    name = {n: idx[frozenset(v)] for n, v in ex["nodes"].items()}
    name["root"] = 0
    for L in ex["links"]:
        t = name[L["node"]]
        assert (out["marked"][t] >> L["l"]) & 1, L
        arr = out["lc"] if L["kind"] == "child" else out["ls"]
        assert int(arr[t][L["l"]]) == name[L["target"]], L
    rows = sorted(map(tuple, out["rows"].tolist()))
    assert rows == sorted(map(tuple, ex["retrieve_t1_l3_with_u0"]))
    ret = sorted(map(tuple, out["retrieved"].tolist()))
    assert ret == sorted(map(tuple, ex["retrieve_t1_l3_with_u0"]))


@pytest.mark.parametrize("seed", [1, 2])
def test_retrieval_matches_brute_force(D, seed):
    """ListingIST(t, k - 1, {root}) from every (k-1)-memoised node of a root's
    trie (random graph, forced ListingDense, k = 4..6) against the
    (k-1)-cliques of the node's vertex set, enumerated in Python."""
    import itertools
    g = gg.gnp(40, 0.7, 300 + seed)
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
    adj = [set(g.col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist()) for v in range(g.n)]
    rank = G.ranks()
    root = int(np.argmin(rank))            # the first vertex: the widest out-neighbourhood
    checked = 0
    for k in (4, 5, 6):
        l = k - 1
        base = D.ist_inspect(G, k, root, cfg=D.config(memo=2))
        loc = [int(v) for v in base["local_ids"]]
        for t, s in enumerate(base["nodes"]):
            if t == 0 or not (base["marked"][t] >> l) & 1:
                continue
            bits = np.zeros(16, np.uint64)
            for i, v in enumerate(loc):
                if v in s:
                    bits[i // 64] |= np.uint64(1 << (i % 64))
            out = D.ist_inspect(G, k, root, cfg=D.config(memo=2), ret_set=bits, ret_l=l)
            got = sorted(map(tuple, out["retrieved"].tolist()))
            want = sorted(tuple(sorted((root,) + c)) for c in itertools.combinations(sorted(s), l)
                          if all(b in adj[a] for a, b in itertools.combinations(c, 2)))
            assert got == want, (k, t, sorted(s))
            checked += 1
    assert checked > 10


def test_device_rows_sink(D, oracle_mod):
    """DIST_LIST_DEVICE_ROWS: the sink receives device pointers; the rows it
    is handed add up to the count, and the fingerprint equals the oracle's."""
    g = gg.turan(50, 7)
    G = D.orient(g.row_ptr, g.col)
    seen = []

    def raw(ptr, n, k):
        seen.append(n)
        return 0

    _, cnt, fp, rc = D.list_cliques(G, 5, cfg=D.config(list_bytes=1 << 22), device_rows=True, raw_sink=raw)
    assert rc == D.OK
    assert (cnt, fp) == oracle_mod.count(g.row_ptr, g.col, 5)
    assert sum(seen) == cnt and len(seen) > 1
