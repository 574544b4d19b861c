"""Parity at full size, in the launch configuration the benchmark times.

The one-large-graph workload (Chung-Lu n = 10^6, exponent 2.2, mean degree
20, cap 5,000, 200 planted K30) has ~5e16 9-cliques: the enumerating oracle
cannot list them, but its pivot-based counter totals every root in under a
minute (tests/golden/cfg2_totals.json, written by make_cfg2_totals.py from
the oracle alone).  Each test compares the benchmark's call (count and
fingerprint) with that total, runs the whole graph again with per-root
output, checks that the per-root results add up to it, and compares seeded
samples of roots one by one: roots whose
search the enumerating oracle finishes quickly (C(d+, k-1) below a bound),
and the dense core (the heaviest roots and a sample of roots with d+ >= 64)
through the oracle's pivot-based counter.

The batched workload (4,096 graphs) is checked on every pair against the
oracle's per-pair results (tests/golden/cfg4_totals.json), and on the
smallest sampled graphs through the enumerating oracle."""
import math

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


@pytest.fixture(scope="module")
def big(D):
    g = gg.large_powerlaw()
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
    # out-degrees under the (degree, id) order, by original id
    deg = np.diff(g.row_ptr).astype(np.int64)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    ks = deg[src] * (g.n + 1) + src
    kd = deg[g.col] * (g.n + 1) + g.col
    outd = np.bincount(src[ks < kd], minlength=g.n)
    return g, G, outd


def _sample_roots(outd, k, bound, n_uniform, n_heavy, seed):
    ok = np.array([d >= k - 1 and math.comb(int(d), k - 1) <= bound for d in outd])
    cand = np.flatnonzero(ok)
    rng = np.random.default_rng(seed)
    pick = set(rng.choice(cand, size=min(n_uniform, len(cand)), replace=False).tolist())
    heavy = cand[np.argsort(-outd[cand], kind="stable")[:n_heavy]]
    pick.update(int(x) for x in heavy)
    return np.array(sorted(pick), dtype=np.int32)


def _golden_totals():
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cfg2_totals.json")))


@pytest.mark.parametrize("k,fp,bound", [(5, 1, 2e7), (7, 1, 2e6), (9, 1, 2e6)])
def test_large_graph_sampled_roots(D, oracle_mod, big, k, fp, bound):
    g, G, outd = big
    cfg = D.config(fingerprint=fp)
    print("full-size k=%d fp=%d" % (k, fp), flush=True)
    total, tfp, rc = D.count(G, k, cfg=cfg)          # the benchmark's call
    assert rc == D.OK
    # the whole-graph total and fingerprint, against the oracle's (every root
    # through the pivot-based counter; tests/golden/make_cfg2_totals.py)
    gold = _golden_totals()
    assert (gold["n"], gold["m"]) == (g.n, g.m)
    assert (total, tfp) == (int(gold["results"][str(k)]["count"]), int(gold["results"][str(k)]["fp"]))
    per = np.zeros(3 * g.n, np.uint64)
    total2, tfp2, rc2 = D.count(G, k, cfg=cfg, per_root=per)
    assert (total2, tfp2, rc2) == (total, tfp, rc)
    lo = per[0::3].astype(object)
    hi = per[1::3].astype(object)
    assert int(sum(lo)) + (int(sum(hi)) << 64) == total
    if fp:
        P61 = (1 << 61) - 1
        assert sum(int(x) for x in per[2::3]) % P61 == tfp

    def check(roots, want):
        for v, (wc, wf) in zip(roots, want):
            got_c = int(per[3 * v]) | (int(per[3 * v + 1]) << 64)
            assert got_c == wc, (int(v), int(outd[v]))
            if fp:
                assert int(per[3 * v + 2]) == wf, int(v)

    # roots the plain oracle enumerates quickly
    roots = _sample_roots(outd, k, bound, 3000, 40, 100 + k)
    print("  %d enumerable roots, heaviest d+ = %d" % (len(roots), int(outd[roots].max())), flush=True)
    check(roots, oracle_mod.count_roots(g.row_ptr, g.col, k, roots))
    # the dense core: the 64 heaviest roots and 100 more with d+ >= 64, by
    # the pivot-based reference (pinned against the enumerating oracle)
    order = np.argsort(-outd, kind="stable")
    rng = np.random.default_rng(200 + k)
    mid = np.flatnonzero(outd >= 64)
    heavy = np.unique(np.concatenate([order[:64], rng.choice(mid, size=min(100, len(mid)), replace=False)]))
    heavy = heavy.astype(np.int32)
    print("  %d dense-core roots, d+ up to %d" % (len(heavy), int(outd[heavy].max())), flush=True)
    want = oracle_mod.pivot_count_roots(g.row_ptr, g.col, k, heavy)
    check(heavy, want)
    print("  sampled roots hold %.3g of %.3g cliques" % (
        sum(c for c, _ in want), float(total)), flush=True)


def test_batched_workload_every_pair(D, oracle_mod):
    """Every pair of the full 4,096-pair batch, graph-captured as the
    benchmark runs it, against the oracle: the digest of the per-pair
    (count, fp) list, their sums and the first 256 pairs verbatim, written by
    tests/golden/make_cfg4_totals.py from the oracle's pivot-based counter;
    the 40 smallest graphs of a seeded sample also against the enumerating
    oracle."""
    import json
    import os
    sys_path = os.path.join(os.path.dirname(__file__), "golden")
    gold = json.load(open(os.path.join(sys_path, "cfg4_totals.json")))
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_cfg4_totals", os.path.join(sys_path, "make_cfg4_totals.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    specs = gg.batch_specs()
    graphs = gg.batch_graphs(specs)
    ks = [s["k"] for s in specs]
    assert (len(specs), sum(g.m for g in graphs)) == (gold["pairs"], gold["edges"])
    G = [D.orient(g.row_ptr, g.col) for g in graphs]
    res, rc, ms = D.count_batch(G, ks, cfg=D.config(), use_graph=True)
    assert rc in (D.OK, D.E_OVERFLOW)
    P61 = (1 << 61) - 1
    print("batched: %d pairs in %.1f ms" % (len(res), ms), flush=True)
    for i, (c, f) in enumerate(gold["first"]):
        assert res[i] == (int(c), int(f)), i
    assert str(sum(c for c, _ in res)) == gold["sum_count"]
    assert str(sum(f for _, f in res) % P61) == gold["sum_fp"]
    assert mk.pair_digest(res) == gold["sha256"]
    rng = np.random.default_rng(44)
    sample = sorted(rng.choice(len(specs), size=300, replace=False).tolist())
    for i in sorted(sample, key=lambda i: specs[i]["n"])[:40]:
        g = graphs[i]
        assert res[i] == oracle_mod.count(g.row_ptr, g.col, ks[i]), i
    # a replay of the captured launch gives the same results for every pair
    res2, rc2, _ = D.count_batch(G, ks, cfg=D.config(), use_graph=True)
    assert res2 == res
    for Gi in G:
        Gi.free()


@pytest.fixture(scope="module")
def rmat():
    return gg.dense_core_rmat()


def test_dense_core_rmat_orientation_and_budget(D, rmat):
    """The dense-core stress graph (R-MAT scale 22, 64M edges): degeneracy
    order bounds every out-degree by the degeneracy the oracle computes
    (stored by tests/golden/make_rmat_degeneracy.py); both orders keep every
    root within the widest (1024-bit) class; a search of its ~1000-wide dense
    core is cut off cleanly by a deadline in either order (an exact count at
    k >= 6 is beyond a search here)."""
    import json
    import os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rmat_s22_degeneracy.json")))
    g = rmat
    assert (g.n, g.m) == (fx["n"], fx["m"])
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGENERACY)
    info = G.info()
    assert info.order_bound == fx["degeneracy"]
    assert info.max_outdeg <= fx["degeneracy"] <= 1024
    assert np.array_equal(np.sort(G.ranks()), np.arange(g.n))
    H = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
    assert fx["degeneracy"] <= H.info().max_outdeg <= 1024
    for X in (G, H):
        with pytest.raises(D.DistError) as e:
            D.count(X, 6, cfg=D.config(fingerprint=0, deadline_ms=3000))
        assert e.value.status == D.E_CANCELLED


def test_dense_core_rmat_k6_counted(D, oracle_mod, rmat, capsys):
    """k = 6 on the dense-core graph in degree order, which the heavy roots'
    arcs as EdgeParallel units bring within about two minutes: the total and
    fingerprint equal the sum of the per-root results; roots the enumerating
    oracle finishes quickly and mid-size roots (64 <= d+ < 512, through the
    oracle's pivot-based counter) equal the oracle's one by one.  The ~9,000
    roots of d+ >= 512 (the dense core) are beyond the CPU oracle: parity
    unpinned there."""
    def step(msg):
        # each finished step is reported as it ends (the test runs minutes)
        with capsys.disabled():
            print("  [dense core k=6] " + msg, flush=True)

    g = rmat
    k = 6
    G = D.orient(g.row_ptr, g.col, order=D.ORDER_DEGREE)
    per = np.zeros(3 * g.n, np.uint64)
    step("oriented; counting with per-root output (about two minutes)")
    total, tfp, rc = D.count(G, k, cfg=D.config(deadline_ms=300000), per_root=per)
    assert rc == D.OK
    step("counted: %d" % total)
    lo = per[0::3].astype(object)
    hi = per[1::3].astype(object)
    assert int(sum(lo)) + (int(sum(hi)) << 64) == total
    P61 = (1 << 61) - 1
    assert sum(int(x) for x in per[2::3]) % P61 == tfp
    deg = np.diff(g.row_ptr).astype(np.int64)
    src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    ks = deg[src] * (g.n + 1) + src
    kd = deg[g.col] * (g.n + 1) + g.col
    outd = np.bincount(src[ks < kd], minlength=g.n)

    def check(roots, want):
        for v, (wc, wf) in zip(roots, want):
            assert int(per[3 * v]) | (int(per[3 * v + 1]) << 64) == wc, (int(v), int(outd[v]))
            assert int(per[3 * v + 2]) == wf, int(v)

    roots = _sample_roots(outd, k, 2e6, 2000, 0, 300 + k)
    check(roots, oracle_mod.count_roots(g.row_ptr, g.col, k, roots))
    step("%d enumerable roots equal the oracle's" % len(roots))
    rng = np.random.default_rng(400 + k)
    mid = np.concatenate([rng.choice(np.flatnonzero((outd >= a) & (outd < b)), 12, replace=False)
                          for a, b in ((64, 128), (128, 256), (256, 512))]).astype(np.int32)
    check(mid, oracle_mod.pivot_count_roots(g.row_ptr, g.col, k, mid))
    step("%d mid-size roots equal the oracle's pivot-based counts" % len(mid))
