"""Definitions written out in plain Python for pinning the oracle.

Nothing here calls the oracle or the HIP path.  Each function is the plain
mathematical definition of a quantity (a brute-force enumeration, a closed
form or a textbook identity) so that the C oracle can be checked against
something other than itself.
"""
from __future__ import annotations

import itertools
from math import comb

import numpy as np

P61 = (1 << 61) - 1
MASK64 = (1 << 64) - 1


def g(v: int) -> int:
    """Fingerprint weight: 1 + (one SplitMix64 step from 0x44495354 ^ v)
    mod (2^61 - 2).  SplitMix64 (Steele, Lea, Flood 2014): add the golden
    gamma 0x9E3779B97F4A7C15, then z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
    z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31."""
    z = ((0x44495354 ^ v) + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    z = z ^ (z >> 31)
    return 1 + z % (P61 - 1)


def adjacency_sets(row_ptr, col):
    n = len(row_ptr) - 1
    return [set(int(x) for x in col[row_ptr[u]:row_ptr[u + 1]]) for u in range(n)]


def brute_cliques(row_ptr, col, k):
    """Every k-subset whose members are pairwise adjacent (definition)."""
    adj = adjacency_sets(row_ptr, col)
    n = len(adj)
    out = []
    for c in itertools.combinations(range(n), k):
        if all(c[j] in adj[c[i]] for i in range(k) for j in range(i + 1, k)):
            out.append(c)
    return out


def fingerprint(cliques) -> int:
    s = 0
    for c in cliques:
        p = 1
        for v in c:
            p = p * g(int(v)) % P61
        s = (s + p) % P61
    return s


def elementary_symmetric(values, k) -> int:
    """e_k(values) mod p by the standard O(n k) recurrence."""
    e = [1] + [0] * k
    for x in values:
        for j in range(k, 0, -1):
            e[j] = (e[j] + e[j - 1] * x) % P61
    return e[k]


def complete_graph_result(n, k):
    """K_n: C(n, k) cliques; fp = e_k(g(0..n-1))."""
    return comb(n, k), elementary_symmetric([g(v) for v in range(n)], k)


def turan_result(n, r, k):
    """Complete r-partite T(n, r), part of v = v mod r.  A k-clique takes at
    most one vertex per part, so count = sum over k-subsets of parts of the
    product of part sizes, and fp = e_k(S_1..S_r) with S_i = sum of g over
    part i."""
    sizes = [len(range(p, n, r)) for p in range(r)]
    q, a = divmod(n, r)
    count = sum(comb(a, j) * comb(r - a, k - j) * (q + 1) ** j * q ** (k - j)
                for j in range(0, k + 1))
    direct = 0
    for s in itertools.combinations(range(r), k):
        prod = 1
        for i in s:
            prod *= sizes[i]
        direct += prod
    assert count == direct
    S = [sum(g(v) for v in range(p, n, r)) % P61 for p in range(r)]
    return count, elementary_symmetric(S, k)


def triangles_by_trace(row_ptr, col) -> int:
    """Number of triangles = trace(A^3) / 6."""
    n = len(row_ptr) - 1
    A = np.zeros((n, n), dtype=np.int64)
    for u in range(n):
        A[u, col[row_ptr[u]:row_ptr[u + 1]]] = 1
    return int(np.trace(A @ A @ A)) // 6


def degeneracy_by_definition(row_ptr, col) -> int:
    """max over nonempty vertex subsets S of the minimum degree of G[S]."""
    adj = adjacency_sets(row_ptr, col)
    n = len(adj)
    best = 0
    for mask in range(1, 1 << n):
        S = [v for v in range(n) if mask >> v & 1]
        Sset = set(S)
        md = min(len(adj[v] & Sset) for v in S)
        best = max(best, md)
    return best


def soft_embeddable(out, x, i, memo=None) -> bool:
    """Is there a soft embedding of an i-tree rooted at x in the DAG ``out``
    (out[x] = out-neighbours, the order is the integer order)?

    An i-tree's root has children that are a 1-tree, 2-tree, ..., (i-1)-tree
    with out-degrees 0, 1, ..., i-2; arcs must map to arcs, and a sibling of
    smaller out-degree must map to a larger vertex, so the images y_1 > y_2
    > ... > y_{i-1} are out-neighbours of x with y_j the root of an embedded
    j-tree.  Subtrees embed independently (the map need not be injective).
    Exhaustive search over such chains."""
    if memo is None:
        memo = {}
    key = (x, i)
    if key in memo:
        return memo[key]
    if i == 1:
        memo[key] = True
        return True
    nbrs = sorted(out[x], reverse=True)

    def chain(start, j):
        if j == i:
            return True
        for t in range(start, len(nbrs)):
            y = nbrs[t]
            if soft_embeddable(out, y, j, memo) and chain(t + 1, j + 1):
                return True
        return False

    res = chain(0, 1)
    memo[key] = res
    return res


def max_soft_embedding(out, x, cap=64) -> int:
    """Maximum l with a soft embedding of an l-tree rooted at x."""
    memo = {}
    l = 1
    while l < cap and soft_embeddable(out, x, l + 1, memo):
        l += 1
    return l


def is_soft_embedding(arcs, children, f) -> bool:
    """Check the two conditions of the definition of a soft embedding for a
    rooted tree given by ``children`` (node -> list of child nodes)."""
    arcset = set(map(tuple, arcs))

    def deg(v):
        return len(children.get(v, []))

    for v, cs in children.items():
        for c in cs:
            if (f[v], f[c]) not in arcset:
                return False
        for a in cs:
            for b in cs:
                if deg(a) < deg(b) and not f[a] > f[b]:
                    return False
    return True
