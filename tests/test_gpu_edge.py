"""EdgeParallel work units (Section VII-D): with edge_units = W every root
whose subgraph takes at least W words is searched as one unit per arc (u, v),
over G[N+(u) & N+(v)] for (k - 2)-cliques.  Per-root results (the units of
a root add into its slot) and totals must equal the oracle's under every
switch: memo 0/1/2, pruning on and off, fingerprints on and off, the
arc's children shared by several units (sub_units), and whole roots split
into child ranges beside the arcs (chunk_work)."""
import numpy as np
import pytest

from paper_2502_00317_amd import graphgen as gg

pytestmark = pytest.mark.gpu

P61 = (1 << 61) - 1


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    from paper_2502_00317_amd import dist
    dist.lib()
    return dist


def _planted(n, p, s, seed):
    """G(n, p) plus one planted clique on s random vertices."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(len(iu)) < p
    a, b = iu[keep], ju[keep]
    plant = np.sort(rng.choice(n, size=s, replace=False))
    pi, pj = np.triu_indices(s, 1)
    e = np.unique(np.stack([np.concatenate([a, plant[pi]]), np.concatenate([b, plant[pj]])], 1), axis=0)
    return gg.csr_from_edges(n, e[:, 0], e[:, 1], name="G(%d,%.2f)+K%d" % (n, p, s))


def _near_complete(n, removed, seed):
    rng = np.random.default_rng(900 + seed)
    iu, ju = np.triu_indices(n, 1)
    keep = np.ones(len(iu), bool)
    keep[rng.choice(len(iu), size=removed, replace=False)] = False
    return gg.csr_from_edges(n, iu[keep], ju[keep], name="K%d-%d" % (n, removed))


def _check(D, oracle_mod, g, ks, cfgs, edge_units=1):
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)  # the oracle's root order
    for k in ks:
        want = oracle_mod.pivot_count_roots(g.row_ptr, g.col, k, np.arange(g.n, dtype=np.int32))
        for cfg in cfgs:
            for fp in (1, 0):
                print("edge units", edge_units, g.name, k, cfg, fp, flush=True)
                per = np.zeros(3 * max(g.n, 1), np.uint64)
                c, f, rc = D.count(G, k, cfg=D.config(edge_units=edge_units, fingerprint=fp, **cfg), per_root=per)
                assert rc == D.OK
                got = [int(per[3 * v]) | (int(per[3 * v + 1]) << 64) for v in range(g.n)]
                assert got == [w for w, _ in want], (g.name, k, cfg, fp)
                assert c == sum(w for w, _ in want)
                if fp:
                    assert [int(per[3 * v + 2]) for v in range(g.n)] == [x for _, x in want], (g.name, k, cfg)
                    assert f == sum(x for _, x in want) % P61
                else:
                    assert f == 0


CFGS = [dict(memo=1, prune=1), dict(memo=0, prune=0), dict(memo=2, prune=1),
        dict(memo=1, prune=1, chunk_work=64), dict(memo=2, prune=0, sub_units=3)]


def test_fig2(D, oracle_mod):
    _check(D, oracle_mod, gg.fig2(), range(1, 8), CFGS)


@pytest.mark.parametrize("seed", range(4))
def test_random(D, oracle_mod, seed):
    rng = np.random.default_rng(40 + seed)
    n = int(rng.integers(20, 90))
    g = gg.gnp(n, float(rng.uniform(0.3, 0.8)), 800 + seed)
    _check(D, oracle_mod, g, (3, 4, 5, 6, 8), CFGS)


def test_planted_and_nearly_complete(D, oracle_mod):
    """Complete and nearly complete arc sets take the closed forms in the
    arc's own first frame; with several units per arc only the first counts
    them."""
    for g in (_planted(150, 0.3, 40, 11), _near_complete(50, 4, 0), _near_complete(70, 9, 1), gg.complete(30)):
        _check(D, oracle_mod, g, (4, 5, 7, 9), CFGS)


def _blocks(n, p, blocks, seed):
    """Sparse uniform edges plus dense random blocks (size, density): roots
    of one to three words of out-neighbours."""
    rng = np.random.default_rng(seed)
    m = int(p * n * (n - 1) / 2)
    A, B = [rng.integers(0, n, m)], [rng.integers(0, n, m)]
    for s, q in blocks:
        vs = rng.choice(n, size=s, replace=False)
        iu, ju = np.triu_indices(s, 1)
        keep = rng.random(len(iu)) < q
        A.append(vs[iu[keep]])
        B.append(vs[ju[keep]])
    a, b = np.concatenate(A), np.concatenate(B)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    e = np.unique(np.stack([lo[lo != hi], hi[lo != hi]], 1), axis=0)
    return gg.csr_from_edges(n, e[:, 0], e[:, 1], name="blocks")


def test_mixed_classes(D, oracle_mod):
    """Only the wider roots are split (edge_units = 2, 3): their arcs share the
    width classes with whole roots of the same launch."""
    g = _blocks(3000, 0.004, [(320, 0.55), (220, 0.7), (150, 0.85)], 5)
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
    assert G.info().max_outdeg > 128
    for ew in (2, 3):
        _check(D, oracle_mod, g, (4, 5), CFGS[:3], edge_units=ew)


@pytest.mark.parametrize("n,r,ks", [(700, 700, (4, 6)), (700, 35, (4, 5))])
def test_wide_roots(D, n, r, ks):
    """Roots of 513..1023 out-neighbours (16-word rows) split into arcs:
    complete and Turan graphs against their closed forms."""
    import refdefs as R
    g = gg.complete(n) if r == n else gg.turan(n, r)
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
    for k in ks:
        want = R.complete_graph_result(n, k) if r == n else R.turan_result(n, r, k)
        for ew in (4, 16):
            print("wide edge units", n, r, k, ew, flush=True)
            c, f, rc = D.count(G, k, cfg=D.config(edge_units=ew, deadline_ms=60000))
            assert rc in (D.OK, D.E_OVERFLOW)
            assert (c, f) == want, (n, r, k, ew)


def test_ignored_cases(D, oracle_mod):
    """k < 4 and the shared trie run without edge units; the results are the
    same either way."""
    g = gg.gnp(60, 0.5, 3)
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
    for k in (1, 2, 3, 5):
        want = oracle_mod.count(g.row_ptr, g.col, k)
        for cfg in (dict(edge_units=1), dict(edge_units=1, trie_tau=64), dict(edge_units=-1)):
            c, f, rc = D.count(G, k, cfg=D.config(**cfg))
            assert rc == D.OK and (c, f) == want, (k, cfg)
