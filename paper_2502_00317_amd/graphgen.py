"""Seeded synthetic graph generators (inputs only).

This module holds none of the clique-listing arithmetic.  It produces simple
undirected graphs in CSR form (``row_ptr`` int32[n+1], ``col`` int32[2m],
rows sorted ascending, symmetric, no self-loops, no duplicates) for the test
suite, the benchmark and the serving replay.  Both the HIP path and the CPU
oracle consume its output; neither is imported here.

The paper measures on real networks (Table 3: social, web and mesh graphs
with power-law degrees, degeneracy 29..1,120 and maximum clique 24..428).
Those datasets are not available, so seeded synthetic graphs of the same
shape stand in for them:

* Chung-Lu graphs with a power-law expected-degree sequence: edge {i, j}
  present independently with probability min(1, w_i w_j / sum(w)).  Sampled
  with the skip method of Miller and Hagberg (2011) over weights sorted in
  descending order, vectorised across all source vertices at once.
* R-MAT graphs (Chakrabarti, Zhan, Faloutsos 2004): each edge picks one of
  four quadrants per level with probabilities (a, b, c, d).
* Planted cliques: s distinct uniform vertices made pairwise adjacent.
* Closed-form families for pins: complete graphs, Turan graphs, G(n, p),
  disjoint unions, relabelings, and the worked example of Figure 2.

Random numbers come from NumPy's PCG64 through ``SeedSequence`` so every
graph is reproducible from its seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Graph:
    """Undirected simple graph in CSR form."""

    row_ptr: np.ndarray
    col: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(len(self.row_ptr) - 1)

    @property
    def m(self) -> int:
        return int(len(self.col) // 2)

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def csr_from_edges(n: int, u, v, name: str = "", meta=None) -> Graph:
    """Symmetrise, drop self-loops and duplicates, sort rows."""
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    keep = u != v
    u, v = u[keep], v[keep]
    if len(u) and (u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n):
        raise ValueError("edge endpoint out of range")
    keys = np.concatenate([u * n + v, v * n + u])
    keys = np.unique(keys)
    rows = keys // n
    cols = (keys % n).astype(np.int32)
    counts = np.bincount(rows, minlength=n) if n > 0 else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return Graph(row_ptr.astype(np.int32), cols, name, dict(meta or {}))


def edges_of(g: Graph):
    """Each undirected edge once, as (u, v) with u < v."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    cols = g.col.astype(np.int64)
    keep = rows < cols
    return rows[keep], cols[keep]


# ---- closed-form families -------------------------------------------------

def empty(n: int) -> Graph:
    return csr_from_edges(n, [], [], name="empty%d" % n)


def complete(n: int) -> Graph:
    iu, ju = np.triu_indices(n, 1)
    return csr_from_edges(n, iu, ju, name="K%d" % n)


def turan(n: int, r: int) -> Graph:
    """Complete r-partite graph with parts as equal as possible; vertex v
    belongs to part v mod r."""
    iu, ju = np.triu_indices(n, 1)
    keep = (iu % r) != (ju % r)
    return csr_from_edges(n, iu[keep], ju[keep], name="T(%d,%d)" % (n, r),
                          meta={"parts": [list(range(p, n, r)) for p in range(r)]})


def gnp(n: int, p: float, seed: int) -> Graph:
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(len(iu)) < p
    return csr_from_edges(n, iu[keep], ju[keep], name="G(%d,%.3f)#%d" % (n, p, seed))


def disjoint_union(*gs: Graph) -> Graph:
    us, vs, off = [], [], 0
    for g in gs:
        u, v = edges_of(g)
        us.append(u + off)
        vs.append(v + off)
        off += g.n
    return csr_from_edges(off, np.concatenate(us) if us else [],
                          np.concatenate(vs) if vs else [], name="union")


def relabel(g: Graph, perm) -> Graph:
    """Vertex v of g becomes perm[v]."""
    perm = np.asarray(perm, dtype=np.int64)
    u, v = edges_of(g)
    return csr_from_edges(g.n, perm[u], perm[v], name=g.name + "/relabel")


# The DAG of Figure 2(b), vertices u0..u8 in the total order u0 < ... < u8,
# read off the identifying strings of Table 2 (each string lists the
# out-neighbourhood of the clique beside it, in descending order) together
# with the statement in Section I that N(u1) = N(u0).
FIG2_OUT = {
    0: [2, 3, 4, 5, 7],
    1: [2, 3, 4, 5, 7],
    2: [3, 4, 7, 8],
    3: [6, 7, 8],
    4: [5, 6, 7, 8],
    5: [6, 7, 8],
    6: [7, 8],
    7: [8],
    8: [],
}


def fig2() -> Graph:
    us = [u for u, vs in FIG2_OUT.items() for _ in vs]
    vs = [v for u, vv in FIG2_OUT.items() for v in vv]
    return csr_from_edges(9, us, vs, name="fig2")


# ---- power-law Chung-Lu ----------------------------------------------------

def powerlaw_weights(n: int, gamma: float, dbar: float, cap: float | None) -> np.ndarray:
    """Deterministic power-law expected degrees, descending:
    w_i = c * (n / (i + 1)) ** (1 / (gamma - 1)), clipped at ``cap``, with c
    found by bisection so that the clipped mean equals ``dbar``."""
    base = (n / np.arange(1, n + 1, dtype=np.float64)) ** (1.0 / (gamma - 1.0))
    cap = float(n - 1) if cap is None else float(min(cap, n - 1))

    def mean_at(c):
        return float(np.minimum(c * base, cap).mean())

    lo, hi = 0.0, 1.0
    while mean_at(hi) < dbar:
        hi *= 2.0
        if hi > 1e12:
            raise ValueError("mean degree %.3f unreachable under cap %.1f" % (dbar, cap))
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if mean_at(mid) < dbar:
            lo = mid
        else:
            hi = mid
    return np.minimum(hi * base, cap)


def chung_lu_sorted(w: np.ndarray, rng: np.random.Generator):
    """Edges (i, j), i < j, of the Chung-Lu model over indices of the
    descending weight vector ``w``: P[{i,j}] = min(1, w_i w_j / S).

    Skip sampling (Miller and Hagberg 2011): for source i the candidate
    probability is non-increasing in j, so from the current bound p the
    next candidate is reached by a geometric jump and accepted with
    probability q/p, where q is the true probability there.  All sources
    advance together, one proposal per source per round."""
    n = len(w)
    S = float(w.sum())
    if n < 2 or S <= 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    u = np.arange(n - 1, dtype=np.int64)
    v = u + 1
    p = np.minimum(w[u] * w[v] / S, 1.0)
    live = p > 0
    u, v, p = u[live], v[live], p[live]
    out_u, out_v = [], []
    while len(u):
        r = rng.random(len(u))
        skip = np.zeros(len(u), dtype=np.int64)
        lt = p < 1.0
        if lt.any():
            jump = np.floor(np.log1p(-r[lt]) / np.log1p(-p[lt]))
            skip[lt] = np.minimum(jump, float(n)).astype(np.int64)
        v = v + skip
        live = v < n
        u, v, p = u[live], v[live], p[live]
        if not len(u):
            break
        q = np.minimum(w[u] * w[v] / S, 1.0)
        r2 = rng.random(len(u))
        acc = r2 * p < q
        out_u.append(u[acc])
        out_v.append(v[acc])
        p = q
        v = v + 1
        live = (v < n) & (p > 0)
        u, v, p = u[live], v[live], p[live]
    if not out_u:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(out_u), np.concatenate(out_v)


def plant_edges(n: int, sizes, rng: np.random.Generator):
    """All pairs inside each planted clique of s distinct uniform vertices."""
    us, vs = [], []
    for s in sizes:
        s = int(min(s, n))
        if s < 2:
            continue
        verts = rng.choice(n, size=s, replace=False).astype(np.int64)
        iu, ju = np.triu_indices(s, 1)
        us.append(verts[iu])
        vs.append(verts[ju])
    if not us:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(us), np.concatenate(vs)


def chung_lu(n: int, gamma: float, dbar: float, cap: float | None, seed,
             plants=(), name: str = "") -> Graph:
    """Power-law Chung-Lu graph plus planted cliques of the given sizes."""
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    s_perm, s_edges, s_plant = ss.spawn(3)
    w = powerlaw_weights(n, gamma, dbar, cap)
    perm = np.random.default_rng(s_perm).permutation(n).astype(np.int64)
    i, j = chung_lu_sorted(w, np.random.default_rng(s_edges))
    pu, pv = plant_edges(n, plants, np.random.default_rng(s_plant))
    u = np.concatenate([perm[i], pu])
    v = np.concatenate([perm[j], pv])
    meta = {"model": "chung-lu", "n": n, "gamma": gamma, "dbar": dbar,
            "cap": cap, "plants": list(map(int, plants))}
    return csr_from_edges(n, u, v, name=name or "CL(n=%d)" % n, meta=meta)


# ---- R-MAT -----------------------------------------------------------------

def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed,
         plants=(), name: str = "", chunk: int = 1 << 22) -> Graph:
    """R-MAT with 2^scale vertices and edge_factor * 2^scale draws, one
    quadrant choice per level, no noise; self-loops and duplicates dropped,
    symmetrised, vertex ids scrambled by a seeded permutation."""
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    s_draw, s_perm, s_plant = ss.spawn(3)
    n = 1 << scale
    E = edge_factor * n
    rng = np.random.default_rng(s_draw)
    ab, abc = a + b, a + b + c
    keys = []
    for start in range(0, E, chunk):
        cnt = min(chunk, E - start)
        u = np.zeros(cnt, dtype=np.int64)
        v = np.zeros(cnt, dtype=np.int64)
        for _ in range(scale):
            r = rng.random(cnt)
            ubit = r >= ab
            vbit = ((r >= a) & (r < ab)) | (r >= abc)
            u = (u << 1) | ubit
            v = (v << 1) | vbit
        keep = u != v
        lo = np.minimum(u[keep], v[keep])
        hi = np.maximum(u[keep], v[keep])
        keys.append(np.unique(lo * n + hi))
    keys = np.unique(np.concatenate(keys))
    perm = np.random.default_rng(s_perm).permutation(n).astype(np.int64)
    u = perm[keys // n]
    v = perm[keys % n]
    pu, pv = plant_edges(n, plants, np.random.default_rng(s_plant))
    meta = {"model": "rmat", "scale": scale, "edge_factor": edge_factor,
            "abcd": [a, b, c, 1 - a - b - c], "plants": list(map(int, plants))}
    return csr_from_edges(n, np.concatenate([u, pu]), np.concatenate([v, pv]),
                          name=name or "RMAT(%d)" % scale, meta=meta)


# ---- the benchmark workloads ---------------------------------------------

def small_powerlaw(seed: int = 1) -> Graph:
    """Chung-Lu n=10,000, exponent 2.5, mean degree 8, capped at 200, plus
    20 planted 12-cliques (the small plain-method workload, k = 4)."""
    return chung_lu(10_000, 2.5, 8.0, 200.0, seed, plants=[12] * 20,
                    name="CL n=1e4 g=2.5 d=8 cap=200 +20xK12")


def large_powerlaw(seed: int = 2, n: int = 1_000_000, plants: int = 200) -> Graph:
    """Chung-Lu n=1,000,000, exponent 2.2, mean degree 20, capped at 5,000,
    plus 200 planted 30-cliques (the one-large-graph workload, k = 5, 7, 9).
    ``n`` and ``plants`` may be reduced for quick parity runs."""
    return chung_lu(n, 2.2, 20.0, 5000.0, seed, plants=[30] * plants,
                    name="CL n=%d g=2.2 d=20 cap=5000 +%dxK30" % (n, plants))


def dense_core_rmat(seed: int = 3, scale: int = 22) -> Graph:
    """R-MAT scale 22, edge factor 16, (0.57, 0.19, 0.19, 0.05), plus 10
    planted 60-cliques (the dense-core stress workload, k = 6, 8, 10, 12)."""
    return rmat(scale, 16, 0.57, 0.19, 0.19, seed, plants=[60] * 10,
                name="RMAT s=%d ef=16 +10xK60" % scale)


def batch_specs(seed: int = 4, count: int = 4096):
    """Parameters of the batched workload: per graph n ~ U{50..5000},
    exponent ~ U[2.1, 3.0], mean degree ~ U[4, 40] (clipped to n-1),
    0..3 planted cliques of size ~ U{8..25}, k ~ U{3..12}."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    specs = []
    for i in range(count):
        n = int(rng.integers(50, 5001))
        gamma = float(rng.uniform(2.1, 3.0))
        dbar = float(min(rng.uniform(4.0, 40.0), 0.5 * (n - 1)))
        nplant = int(rng.integers(0, 4))
        plants = [int(x) for x in rng.integers(8, 26, size=nplant)]
        k = int(rng.integers(3, 13))
        specs.append({"i": i, "n": n, "gamma": gamma, "dbar": dbar,
                      "plants": plants, "k": k, "seed": [seed, i]})
    return specs


def batch_graph(spec) -> Graph:
    return chung_lu(spec["n"], spec["gamma"], spec["dbar"], None,
                    np.random.SeedSequence(spec["seed"]), plants=spec["plants"],
                    name="batch#%d" % spec["i"])


def _batch_graph_arrays(spec):
    g = batch_graph(spec)
    return g.row_ptr, g.col


def spec_graph(spec) -> Graph:
    """Chung-Lu graph of a pool / ad-hoc spec (no degree cap beyond n - 1)."""
    return chung_lu(spec["n"], spec["gamma"], spec["dbar"], None,
                    np.random.SeedSequence(spec["seed"]), plants=spec.get("plants", []),
                    name="spec#%d" % spec["i"])


def _spec_graph_arrays(spec):
    g = spec_graph(spec)
    return g.row_ptr, g.col


def _gpu_in_use() -> bool:
    """True if this process may hold a GPU context (torch initialised it, or
    the library's binding is loaded)."""
    import sys
    t = sys.modules.get("torch")
    if t is not None and t.cuda.is_initialized():
        return True
    d = sys.modules.get("paper_2502_00317_amd.dist")
    return d is not None and getattr(d, "_lib", None) is not None


def _map_procs(fn, items, workers: int, chunksize: int):
    """fn over items in worker processes.  A process that holds no GPU
    context forks its workers (no exec, no helper process left behind);
    one that may hold a GPU context spawns them instead.  The pool is closed
    and joined, so every worker ends normally rather than by a signal.
    Results do not depend on the pool."""
    import multiprocessing as mp
    import os
    if workers <= 0:
        workers = min(16, os.cpu_count() or 1)
    if workers == 1 or len(items) < 4:
        return [fn(x) for x in items]
    ctx = mp.get_context("spawn" if _gpu_in_use() else "fork")
    pool = ctx.Pool(workers)
    try:
        out = pool.map(fn, items, chunksize=chunksize)
    finally:
        pool.close()
        pool.join()
    return out


def spec_graphs(specs, workers: int = 0):
    """spec_graph for every spec, in worker processes."""
    arrays = _map_procs(_spec_graph_arrays, specs, workers, 1)
    return [Graph(rp, col, name="spec#%d" % s["i"]) for (rp, col), s in zip(arrays, specs)]


def batch_graphs(specs, workers: int = 0):
    """batch_graph for every spec, in worker processes.  Each graph depends
    only on its spec."""
    arrays = _map_procs(_batch_graph_arrays, specs, workers, 8)
    return [Graph(rp, col, name="batch#%d" % s["i"]) for (rp, col), s in zip(arrays, specs)]


def serving_pool_specs(seed: int = 5, count: int = 64, n_lo: float = 1e4,
                       n_hi: float = 2e6):
    """Resident pool: n log-uniform in [n_lo, n_hi], exponent U[2.2, 2.8],
    mean degree U[10, 30], no cap beyond n - 1."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0]))
    specs = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        specs.append({"i": i, "n": n, "gamma": float(rng.uniform(2.2, 2.8)),
                      "dbar": float(rng.uniform(10.0, 30.0)), "plants": [],
                      "seed": [seed, 1, i]})
    return specs


def serving_queries(seed: int = 5, count: int = 2000, qps: float = 200.0,
                    pool_size: int = 64, adhoc_frac: float = 0.1,
                    adhoc_n=(1e3, 5e4)):
    """Poisson arrival stream of (graph, k) queries; a fraction are ad-hoc
    uploads of fresh Chung-Lu graphs with n log-uniform in adhoc_n."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 2]))
    t = np.cumsum(rng.exponential(1.0 / qps, size=count))
    out = []
    for i in range(count):
        k = int(rng.integers(3, 13))
        if rng.random() < adhoc_frac:
            n = int(round(math.exp(rng.uniform(math.log(adhoc_n[0]), math.log(adhoc_n[1])))))
            spec = {"i": 10_000 + i, "n": n, "gamma": float(rng.uniform(2.2, 2.8)),
                    "dbar": float(rng.uniform(10.0, 30.0)), "plants": [],
                    "seed": [seed, 3, i]}
            out.append({"t": float(t[i]), "k": k, "adhoc": spec})
        else:
            out.append({"t": float(t[i]), "k": k, "graph": int(rng.integers(0, pool_size))})
    return out
