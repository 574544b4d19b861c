"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Counts are compared bit-exactly (u128) and fingerprints exactly (mod
2^61 - 1).  Every switch of the search (memoisation, pruning, order) must
give the same result.
"""
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


CONFIGS = [dict(memo=1, prune=1), dict(memo=0, prune=0), dict(memo=0, prune=1),
           dict(memo=2, prune=1), dict(memo=2, prune=0), dict(memo=1, prune=1, chunk_work=64)]


def _gpu(D, g, k, order, **cfg):
    G = D.orient(g.row_ptr, g.col, order=order)
    c = D.config(deadline_ms=60000, **cfg)
    cnt, fp, rc = D.count(G, k, cfg=c)
    assert rc in (D.OK, D.E_OVERFLOW)
    return cnt, fp


def test_fig2_all_k(D, oracle_mod):
    g = gg.fig2()
    for order in (D.ORDER_DEGREE, D.ORDER_DEGENERACY, D.ORDER_INPUT):
        for k in range(1, 8):
            want = oracle_mod.count(g.row_ptr, g.col, k)
            for cfg in CONFIGS:
                print("fig2", order, k, cfg, flush=True)
                assert _gpu(D, g, k, order, **cfg) == want, (order, k, cfg)


@pytest.mark.parametrize("seed", range(8))
def test_random_small(D, oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 60))
    p = float(rng.uniform(0.2, 0.9))
    g = gg.gnp(n, p, 500 + seed)
    for k in range(1, 9):
        want = oracle_mod.count(g.row_ptr, g.col, k)
        for order in (D.ORDER_DEGREE, D.ORDER_DEGENERACY):
            for cfg in CONFIGS[:4]:
                print("gnp", seed, n, p, k, order, cfg, flush=True)
                assert _gpu(D, g, k, order, **cfg) == want, (seed, k, order, cfg)


@pytest.mark.parametrize("n", [5, 63, 64, 65, 100, 130, 200])
def test_complete(D, oracle_mod, n):
    """Complete graphs: every root's subgraph is complete; widths 1..4
    words with ragged tails."""
    import refdefs as R
    g = gg.complete(n)
    for k in (2, 3, 4, 5, 6):
        want = R.complete_graph_result(n, k)
        for cfg in CONFIGS[:4] + CONFIGS[5:]:
            print("K", n, k, cfg, flush=True)
            assert _gpu(D, g, k, D.ORDER_DEGREE, **cfg) == want


@pytest.mark.parametrize("n,r,k", [(40, 6, 5), (90, 10, 6), (150, 12, 7), (300, 20, 5)])
def test_turan(D, n, r, k):
    """Turan graphs are dense (criterion (1) holds) and exercise the memo."""
    import refdefs as R
    g = gg.turan(n, r)
    want = R.turan_result(n, r, k)
    for order in (D.ORDER_DEGREE, D.ORDER_DEGENERACY):
        for cfg in CONFIGS:
            print("T", n, r, k, order, cfg, flush=True)
            assert _gpu(D, g, k, order, **cfg) == want


def test_small_powerlaw(D, oracle_mod):
    g = gg.small_powerlaw()
    for k in (3, 4, 5, 6):
        want = oracle_mod.count(g.row_ptr, g.col, k)
        for order in (D.ORDER_DEGREE, D.ORDER_DEGENERACY):
            for cfg in CONFIGS[:4]:
                print("cfg1", k, order, cfg, flush=True)
                assert _gpu(D, g, k, order, **cfg) == want


def test_per_root_degree_order(D, oracle_mod):
    g = gg.gnp(80, 0.5, 3)
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
    for k, cw in ((3, 0), (4, 0), (5, 0), (6, 0), (5, 64), (6, 100)):
        per = np.zeros(3 * g.n, np.uint64)
        D.count(G, k, cfg=D.config(chunk_work=cw), per_root=per)
        want = oracle_mod.count_roots(g.row_ptr, g.col, k, np.arange(g.n))
        got = [(int(per[3 * v]) | (int(per[3 * v + 1]) << 64), int(per[3 * v + 2]))
               for v in range(g.n)]
        assert got == want


def test_orientation_orders(D, oracle_mod):
    g = gg.small_powerlaw()
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
    assert np.array_equal(G.ranks(), oracle_mod.degree_rank(g.row_ptr))
    delta, _ = oracle_mod.degeneracy(g.row_ptr, g.col)
    H = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGENERACY)
    info = H.info()
    assert info.order_bound == delta
    assert info.max_outdeg <= delta
    assert sorted(H.ranks()) == list(range(g.n))


def test_root_soft_embed(D, oracle_mod):
    for seed in range(3):
        g = gg.gnp(40, 0.5, seed)
        G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
        want = oracle_mod.root_soft_embed(g.row_ptr, g.col)
        got = D.root_soft_embed(G, 60)
        assert np.array_equal(got, np.minimum(want, 60))


def test_invalid_inputs(D):
    bad = [
        (np.array([0, 1, 2], np.int32), np.array([0, 0], np.int32)),   # self-loop
        (np.array([0, 1, 1], np.int32), np.array([1], np.int32)),      # asymmetric
        (np.array([0, 2, 4], np.int32), np.array([1, 1, 0, 0], np.int32)),  # duplicate
        (np.array([0, 1, 2], np.int32), np.array([2, 0], np.int32)),   # out of range
        (np.array([0, 3, 2], np.int32), np.array([1, 0], np.int32)),   # bad row_ptr
    ]
    for rp, col in bad:
        with pytest.raises(D.DistError) as e:
            D.orient(rp, col)
        assert e.value.status == D.E_INVALID
    g = gg.fig2()
    G = D.orient(g.row_ptr, g.col)
    for k in (0, -1, 65):
        with pytest.raises(D.DistError):
            D.count(G, k)


def test_empty_graphs(D):
    for n in (0, 1, 7):
        g = gg.empty(n)
        G = D.orient(g.row_ptr, g.col)
        assert D.count(G, 1)[0] == n
        assert D.count(G, 2)[0] == 0
        assert D.count(G, 5)[0] == 0


@pytest.mark.parametrize("n,r,ks", [(700, 700, (3, 4, 6)), (700, 35, (3, 4))])
def test_wide_roots(D, n, r, ks):
    """Roots with 513..1023 out-neighbours (16-word rows, one wavefront per
    CU): complete graphs and Turan graphs against their closed forms."""
    import refdefs as R
    g = gg.complete(n) if r == n else gg.turan(n, r)
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
    assert G.info().max_outdeg > 512
    for k in ks:
        want = R.complete_graph_result(n, k) if r == n else R.turan_result(n, r, k)
        for cfg in (dict(memo=1, prune=1), dict(memo=0, prune=1)):
            print("wide", n, r, k, cfg, flush=True)
            assert _gpu(D, g, k, D.ORDER_DEGREE, **cfg) == want


@pytest.mark.parametrize("n,removed,seed", [(40, 1, 0), (40, 3, 1), (60, 5, 2), (90, 6, 3), (90, 9, 4)])
def test_nearly_complete(D, oracle_mod, n, removed, seed):
    """Complete graphs minus a few edges: candidate sets that miss 1..6 edges
    (counted by inclusion-exclusion without fingerprints) and more (searched),
    against the oracle's pivot-based counter (pinned against enumeration)."""
    rng = np.random.default_rng(700 + seed)
    iu, ju = np.triu_indices(n, 1)
    drop = rng.choice(len(iu), size=removed, replace=False)
    keep = np.ones(len(iu), bool)
    keep[drop] = False
    g = gg.csr_from_edges(n, iu[keep], ju[keep], name="K%d-%d" % (n, removed))
    P61 = (1 << 61) - 1
    for k in (3, 4, 5, 7, 9):
        per = oracle_mod.pivot_count_roots(g.row_ptr, g.col, k, np.arange(n, dtype=np.int32))
        want = (sum(c for c, _ in per), sum(f for _, f in per) % P61)
        for order in (D.ORDER_DEGREE, D.ORDER_DEGENERACY):
            for cfg in (dict(memo=1, prune=1), dict(memo=0, prune=0)):
                print("near", n, removed, k, order, cfg, flush=True)
                G = D.orient(g.row_ptr, g.col, order=order)
                c, f, rc = D.count(G, k, cfg=D.config(fingerprint=0, **cfg))
                assert c == want[0], (k, order, cfg)
                assert _gpu(D, g, k, order, **cfg) == want


def _planted(n, p, s, seed):
    """G(n, p) plus one planted clique on s random vertices."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(len(iu)) < p
    a, b = iu[keep], ju[keep]
    plant = np.sort(rng.choice(n, size=s, replace=False))
    pi, pj = np.triu_indices(s, 1)
    a = np.concatenate([a, plant[pi]])
    b = np.concatenate([b, plant[pj]])
    e = np.unique(np.stack([a, b], 1), axis=0)
    return gg.csr_from_edges(n, e[:, 0], e[:, 1], name="G(%d,%.2f)+K%d" % (n, p, s))


@pytest.mark.parametrize("sub", [2, 3, 7, 32])
def test_sub_units(D, oracle_mod, sub):
    """Depth-1 children shared out among several work units (each takes every
    sub-th surviving depth-2 child): per-root results equal the oracle's for
    every split, with and without memoisation, chunking and fingerprints,
    including complete and nearly complete candidate sets at the split frame."""
    P61 = (1 << 61) - 1
    cases = [(gg.gnp(80, 0.5, 3), (6, 7)), (_planted(150, 0.3, 40, 11), (6, 8))]
    rng = np.random.default_rng(900 + sub)
    iu, ju = np.triu_indices(60, 1)
    keep = np.ones(len(iu), bool)
    keep[rng.choice(len(iu), size=5, replace=False)] = False
    cases.append((gg.csr_from_edges(60, iu[keep], ju[keep], name="K60-5"), (7, 9)))
    for g, ks in cases:
        G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
        for k in ks:
            want = oracle_mod.pivot_count_roots(g.row_ptr, g.col, k, np.arange(g.n, dtype=np.int32))
            for cfg in (dict(memo=1), dict(memo=0), dict(memo=2), dict(memo=1, chunk_work=64)):
                for fp in (1, 0):
                    print("sub", sub, g.name, k, cfg, fp, flush=True)
                    per = np.zeros(3 * g.n, np.uint64)
                    c, f, rc = D.count(G, k, cfg=D.config(sub_units=sub, fingerprint=fp, **cfg), per_root=per)
                    assert rc == D.OK
                    got = [int(per[3 * v]) | (int(per[3 * v + 1]) << 64) for v in range(g.n)]
                    assert got == [w for w, _ in want], (k, cfg, fp)
                    assert c == sum(w for w, _ in want)
                    if fp:
                        assert [int(per[3 * v + 2]) for v in range(g.n)] == [x for _, x in want]
                        assert f == sum(x for _, x in want) % P61


@pytest.mark.parametrize("n,ks", [(20, (16, 17, 18, 19)), (64, (17, 18, 30)), (200, (17, 20))])
def test_large_k_closed_forms(D, n, ks):
    """Complete graphs at k > 16: closed forms whose binomials C(|P|, l) lie
    beyond the precomputed table (l > 16) and are computed exactly in 128
    bits, next to ones inside it, against C(n, k) and e_k."""
    import refdefs as R
    g = gg.complete(n)
    for k in ks:
        want = R.complete_graph_result(n, k)
        for cfg in (dict(memo=1, prune=1), dict(memo=0, prune=0)):
            print("K", n, k, cfg, flush=True)
            assert _gpu(D, g, k, D.ORDER_DEGREE, **cfg) == want


@pytest.mark.parametrize("removed,seed", [(2, 0), (5, 1)])
def test_large_k_nearly_complete(D, oracle_mod, removed, seed):
    """K_22 minus a few edges at k = 12..20: inclusion-exclusion terms with
    binomials inside and beyond the table, against the enumerating oracle."""
    n = 22
    rng = np.random.default_rng(800 + seed)
    iu, ju = np.triu_indices(n, 1)
    keep = np.ones(len(iu), bool)
    keep[rng.choice(len(iu), size=removed, replace=False)] = False
    g = gg.csr_from_edges(n, iu[keep], ju[keep], name="K22-%d" % removed)
    for k in (12, 17, 18, 20):
        want = oracle_mod.count(g.row_ptr, g.col, k)
        for fp in (0, 1):
            print("K22-", removed, k, fp, flush=True)
            G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
            c, f, rc = D.count(G, k, cfg=D.config(fingerprint=fp))
            assert c == want[0], (k, fp)
            if fp:
                assert f == want[1], k


@pytest.mark.parametrize("tau", [1, 64, 1 << 20])
def test_shared_trie(D, oracle_mod, tau):
    """The Induced Subgraph Trie shared by the consecutive roots a wave takes
    (trie_tau = tau: cleared at a root once more than tau nodes were
    inserted, never past 2 tau; nodes keyed by their vertex sets as global
    ranks): per-root results and totals equal the oracle's under memo 1 and
    2, with and without fingerprints and sub-units."""
    P61 = (1 << 61) - 1
    cases = [(gg.fig2(), (3, 4, 5)), (gg.gnp(80, 0.5, 3), (5, 7)), (_planted(150, 0.3, 40, 11), (5, 7)),
             (gg.small_powerlaw(), (4, 6))]
    for g, ks in cases:
        G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
        for k in ks:
            want = oracle_mod.pivot_count_roots(g.row_ptr, g.col, k, np.arange(g.n, dtype=np.int32))
            for cfg in (dict(memo=1), dict(memo=2), dict(memo=2, sub_units=3)):
                for fp in (1, 0):
                    print("shared trie", tau, g.name, k, cfg, fp, flush=True)
                    per = np.zeros(3 * g.n, np.uint64)
                    c, f, rc = D.count(G, k, cfg=D.config(trie_tau=tau, fingerprint=fp, **cfg), per_root=per)
                    assert rc == D.OK
                    got = [int(per[3 * v]) | (int(per[3 * v + 1]) << 64) for v in range(g.n)]
                    assert got == [w for w, _ in want], (k, cfg, fp)
                    assert c == sum(w for w, _ in want)
                    if fp:
                        assert [int(per[3 * v + 2]) for v in range(g.n)] == [x for _, x in want]
                        assert f == sum(x for _, x in want) % P61


def test_shared_trie_crosses_roots(D, oracle_mod):
    """Two roots with the same out-neighbourhood (the situation N(u0) = N(u1)
    of the paper's example): with the shared trie the second root finds the
    nodes the first inserted, so it makes more memo hits than per-root memos
    do, with the same results; the batched form clears the trie between
    graphs, so equal vertex sets of different graphs never match."""
    rng = np.random.default_rng(4)
    iu, ju = np.triu_indices(24, 1)
    keep = rng.random(len(iu)) < 0.7
    a, b = list(iu[keep] + 2), list(ju[keep] + 2)
    for twin in (0, 1):
        a += [twin] * 24
        b += list(range(2, 26))
    g = gg.csr_from_edges(26, a, b, name="twins")
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_INPUT)
    for k in (5, 6, 7):
        want = oracle_mod.count(g.row_ptr, g.col, k)
        hits = {}
        for tau in (0, 1 << 20):
            c, f, rc = D.count(G, k, cfg=D.config(memo=2, trie_tau=tau))
            assert (c, f) == want, (k, tau)
            hits[tau] = G.stats().memo_hits
        print("twins", k, hits, flush=True)
        assert hits[1 << 20] > hits[0], (k, hits)
    # batches: the same vertex ids in different graphs
    g2 = gg.gnp(26, 0.6, 9)
    G2 = D.orient(g2.row_ptr, g2.col, order=D.ORDER_INPUT)
    ks = [6, 6, 5, 7, 6]
    graphs = [G, G2, G, G2, G2]
    srcs = [g, g2, g, g2, g2]
    res, rc, _ = D.count_batch(graphs, ks, cfg=D.config(memo=2, trie_tau=1 << 20))
    assert res == [oracle_mod.count(x.row_ptr, x.col, k) for x, k in zip(srcs, ks)]


@pytest.mark.parametrize("missing", [
    [(0, 1)],                      # one edge
    [(0, 1), (2, 3)],              # two disjoint edges (4 endpoints)
    [(0, 1), (0, 2)],              # two edges sharing a vertex (3 endpoints)
    [(3, 7), (7, 11)],             # the same, sharing the middle vertex
    [(0, 1), (1, 2), (2, 3)],      # a path of three: past the per-lane limit
    [(4, 5), (5, 6), (4, 6)],      # a triangle of three
])
def test_children_missing_few_edges(D, oracle_mod, missing):
    """K_n minus a few edges in set patterns: child sets missing one or two
    edges are counted one per lane by inclusion-exclusion (two edges may
    share an endpoint), three go through frames; per-root results equal the
    oracle's under sub-units (a root frame's shared children count in
    sub-unit 0 only), EdgeParallel units, and memo modes that keep the
    frame order."""
    n = 34
    iu, ju = np.triu_indices(n, 1)
    drop = {tuple(sorted(e)) for e in missing}
    keep = np.array([(int(a), int(b)) not in drop for a, b in zip(iu, ju)])
    g = gg.csr_from_edges(n, iu[keep], ju[keep], name="K%d-%s" % (n, missing))
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
    P61 = (1 << 61) - 1
    for k in (3, 4, 5, 6, 7, 9):
        want = oracle_mod.pivot_count_roots(g.row_ptr, g.col, k, np.arange(n, dtype=np.int32))
        for cfg in (dict(memo=1), dict(memo=0, sub_units=3), dict(memo=2, sub_units=7),
                    dict(memo=0, edge_units=1), dict(memo=1, edge_units=1, sub_units=2)):
            for fp in (1, 0):
                per = np.zeros(3 * n, np.uint64)
                c, f, rc = D.count(G, k, cfg=D.config(fingerprint=fp, **cfg), per_root=per)
                assert rc == D.OK
                got = [int(per[3 * v]) | (int(per[3 * v + 1]) << 64) for v in range(n)]
                assert got == [w for w, _ in want], (missing, k, cfg, fp)
                assert c == sum(w for w, _ in want)
                if fp:
                    assert [int(per[3 * v + 2]) for v in range(n)] == [x for _, x in want], (missing, k, cfg)
                    assert f == sum(x for _, x in want) % P61
