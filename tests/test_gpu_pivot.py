"""Pivot-based counting on the GPU (dist_count_all): the count and
fingerprint of every clique size from one call, against the oracle --
enumeration where it finishes, the oracle's pivot-based counter (pinned
against enumeration) elsewhere, closed forms on complete and Turan graphs,
and the full-size totals of the one-large-graph workload."""
import json
import os

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


def _all(D, g, kmax, order, **cfg):
    G = D.orient(g.row_ptr, g.col, order=order)
    res, rc = D.count_all(G, kmax, cfg=D.config(deadline_ms=120000, **cfg))
    assert rc in (D.OK, D.E_OVERFLOW), rc
    return res, G


def test_fig2_every_k(D, oracle_mod):
    g = gg.fig2()
    for order in (D.ORDER_DEGREE, D.ORDER_DEGENERACY, D.ORDER_INPUT):
        res, _ = _all(D, g, 8, order)
        assert res[0] == (0, 0)
        for k in range(1, 9):
            print("fig2 pivot", order, k, flush=True)
            assert res[k] == oracle_mod.count(g.row_ptr, g.col, k), (order, k)


@pytest.mark.parametrize("seed", range(6))
def test_random_every_k(D, oracle_mod, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 70))
    g = gg.gnp(n, float(rng.uniform(0.2, 0.9)), 900 + seed)
    for order in (D.ORDER_DEGREE, D.ORDER_DEGENERACY):
        res, _ = _all(D, g, 10, order)
        for k in range(1, 11):
            print("gnp pivot", seed, n, order, k, flush=True)
            assert res[k] == oracle_mod.count(g.row_ptr, g.col, k), (seed, k)


def test_closed_forms(D):
    """K_n: C(n, k) and e_k of the weights; Turan T(n, r): the closed form;
    wide roots (K_300: 5-word rows; K_700: 16-word rows) up to k = 16."""
    import refdefs as R
    for n in (20, 64, 65, 300, 700):
        res, _ = _all(D, gg.complete(n), 16, D.ORDER_DEGREE)
        for k in range(1, 17):
            assert res[k] == R.complete_graph_result(n, k), (n, k)
    # (pivoting is exponential on complete multipartite graphs -- their
    # maximal cliques number prod(part sizes) -- so the Turan cases are small)
    for n, r in ((60, 7), (40, 10)):
        res, _ = _all(D, gg.turan(n, r), 16, D.ORDER_DEGREE)
        for k in range(1, 17):
            assert res[k] == R.turan_result(n, r, k), (n, r, k)


def test_powerlaw_every_k_and_per_root(D, oracle_mod):
    """cfg1 (Chung-Lu n = 10^4, planted 12-cliques): every k up to 14 against
    enumeration (k <= 7) and the oracle's pivot counter (k >= 8); per-root
    results at k = 5 against the oracle's per-root counts."""
    g = gg.small_powerlaw()
    res, G = _all(D, g, 14, D.ORDER_DEGREE)
    roots = np.arange(g.n, dtype=np.int32)
    for k in range(1, 15):
        if k <= 7:
            want = oracle_mod.count(g.row_ptr, g.col, k)
        else:
            per = oracle_mod.pivot_count_roots(g.row_ptr, g.col, k, roots)
            want = (sum(c for c, _ in per), sum(f for _, f in per) % P61)
        assert res[k] == want, k
    per = np.zeros(3 * g.n, np.uint64)
    res2, rc = D.count_all(G, 6, per_root=per, per_root_k=5)
    assert rc == D.OK and res2[:7] == res[:7]
    want = oracle_mod.count_roots(g.row_ptr, g.col, 5, roots)
    got = [(int(per[3 * v]) | (int(per[3 * v + 1]) << 64), int(per[3 * v + 2])) for v in range(g.n)]
    assert got == want


@pytest.mark.parametrize("nsub", [2, 3, 7, 64])
def test_split_roots_every_k(D, oracle_mod, nsub):
    """Roots shared by nsub work units (the units deal out the tree nodes at
    depth 2; leaves above count once): every k and the per-root results
    unchanged, against the oracle."""
    for name, g in (("fig2", gg.fig2()), ("gnp", gg.gnp(60, 0.6, 77)), ("turan", gg.turan(40, 10))):
        res, G = _all(D, g, 10, D.ORDER_DEGREE, sub_units=nsub)
        for k in range(1, 11):
            print("split pivot", nsub, name, k, flush=True)
            assert res[k] == oracle_mod.count(g.row_ptr, g.col, k), (nsub, name, k)
    g = gg.small_powerlaw()
    G = D.orient(g.row_ptr, g.col)
    per = np.zeros(3 * g.n, np.uint64)
    res, rc = D.count_all(G, 6, cfg=D.config(sub_units=nsub), per_root=per, per_root_k=5)
    assert rc == D.OK
    for k in range(1, 7):
        assert res[k] == oracle_mod.count(g.row_ptr, g.col, k), (nsub, k)
    want = oracle_mod.count_roots(g.row_ptr, g.col, 5, np.arange(g.n, dtype=np.int32))
    got = [(int(per[3 * v]) | (int(per[3 * v + 1]) << 64), int(per[3 * v + 2])) for v in range(g.n)]
    assert got == want


def test_large_graph_golden_totals(D):
    """The one-large-graph workload (Chung-Lu n = 10^6): one call gives k = 5,
    7 and 9, equal to the oracle's totals (tests/golden/cfg2_totals.json),
    and agrees with the search at k = 3..9."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cfg2_totals.json")))
    g = gg.large_powerlaw()
    assert (g.n, g.m) == (gold["n"], gold["m"])
    res, G = _all(D, g, 9, D.ORDER_DEGREE)
    for k in (5, 7, 9):
        r = gold["results"][str(k)]
        assert res[k] == (int(r["count"]), int(r["fp"])), k
    assert res[2][0] == g.m
    for k in (3, 4, 6, 8):
        c, f, rc = D.count(G, k)
        assert res[k] == (c, f), k


def test_deadline_cancels(D):
    g = gg.gnp(300, 0.9, 3)
    G = D.orient(g.row_ptr, g.col)
    res, rc = D.count_all(G, 16, cfg=D.config(deadline_ms=200))
    assert rc in (D.E_CANCELLED, D.OK, D.E_OVERFLOW)
