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
    for order in (D.ORDER_DEGREE, D.ORDER_DEGENERACY):
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
