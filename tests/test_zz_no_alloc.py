"""dist_count_noalloc (the entry point for callers that cannot allocate
device memory) through the C ABI: its results equal dist_count_ex's with the
same switches, on two calls in a row that share the static scratch block, the
second on a smaller input, and after a call of the allocating entry point."""
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


def _pair(D, g, k, **cfg):
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
    c = D.config(**cfg)
    print("noalloc", g.name, g.n, k, cfg, flush=True)
    want = D.count(G, k, cfg=c)
    got = D.count_noalloc(G, k, cfg=c)
    G.free()
    return got, want


def test_noalloc_equals_count_twice_second_smaller(D):
    big = gg.small_powerlaw()                  # n = 10,000, planted 12-cliques, width classes 1..
    small = gg.gnp(60, 0.5, 11)
    for fp in (1, 0):
        got, want = _pair(D, big, 5, fingerprint=fp)
        assert got == want, ("first call", fp)
        got, want = _pair(D, small, 4, fingerprint=fp)
        assert got == want, ("second, smaller call", fp)


def test_noalloc_wide_roots_and_k1(D):
    """A graph whose roots span several width classes (K_300 minus a few edges:
    5-word rows), then k = 1 and 2 (no search), then a tiny one."""
    n = 300
    rng = np.random.default_rng(5)
    iu, ju = np.triu_indices(n, 1)
    keep = np.ones(len(iu), bool)
    keep[rng.choice(len(iu), size=40, replace=False)] = False
    g = gg.csr_from_edges(n, iu[keep], ju[keep], name="K300-40")
    for k in (6, 1, 2):
        got, want = _pair(D, g, k)
        assert got == want, k
    got, want = _pair(D, gg.fig2(), 4)
    assert got == want and got[0] == 14
