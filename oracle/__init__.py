"""Plain CPU reference for k-clique counting and listing.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import this module; the product library
never does, and the two share no code.

The C library ``liboracle.so`` (built from ``oracle.c`` by ``build()``)
computes the plain definition of the problem (Section II-A, Definition
"k-clique listing"): every k-subset of V whose members are pairwise adjacent,
found by the ordering-based recursive framework of Algorithm 1 with sorted
out-lists intersected by merging.  It reports the count as an unsigned
128-bit integer and the fingerprint

    fp = sum over k-cliques C of prod_{v in C} g(v)  mod (2^61 - 1),
    g(v) = 1 + (splitmix64_next(0x44495354 ^ v) mod (2^61 - 2)).

Every function here is a thin ctypes wrapper; the arithmetic is in oracle.c.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

P61 = (1 << 61) - 1


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_validate.argtypes = [ctypes.c_int32, i32p, i32p]
    lib.oracle_validate.restype = ctypes.c_int
    lib.oracle_weight.argtypes = [ctypes.c_int64]
    lib.oracle_weight.restype = ctypes.c_uint64
    lib.oracle_count.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int,
                                 ctypes.c_int, u64p]
    lib.oracle_count.restype = ctypes.c_int
    lib.oracle_count_roots.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int,
                                       i32p, ctypes.c_int64, ctypes.c_int, u64p]
    lib.oracle_count_roots.restype = ctypes.c_int
    lib.oracle_pivot_count_roots.argtypes = lib.oracle_count_roots.argtypes
    lib.oracle_pivot_count_roots.restype = ctypes.c_int
    lib.oracle_list.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int,
                                i32p, ctypes.c_int64]
    lib.oracle_list.restype = ctypes.c_int64
    lib.oracle_soft_embed.argtypes = [ctypes.c_int32, i32p, i32p, i32p]
    lib.oracle_soft_embed.restype = ctypes.c_int
    lib.oracle_root_soft_embed.argtypes = [ctypes.c_int32, i32p, i32p, i32p]
    lib.oracle_root_soft_embed.restype = ctypes.c_int
    lib.oracle_degeneracy.argtypes = [ctypes.c_int32, i32p, i32p, i32p]
    lib.oracle_degeneracy.restype = ctypes.c_int32
    lib.oracle_degree_rank.argtypes = [ctypes.c_int32, i32p, i32p]
    lib.oracle_degree_rank.restype = ctypes.c_int
    _lib = lib
    return lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _csr(row_ptr, col):
    rp, rpp = _i32(row_ptr)
    c, cp = _i32(col if len(col) else np.zeros(1, np.int32))
    return rp, rpp, c, cp


def validate(row_ptr, col) -> bool:
    rp, rpp, c, cp = _csr(row_ptr, col)
    return _load().oracle_validate(len(rp) - 1, rpp, cp) == 0


def weight(v: int) -> int:
    return int(_load().oracle_weight(int(v)))


def count(row_ptr, col, k: int, nthreads: int = 0):
    """(count as Python int, fp) of all k-cliques."""
    rp, rpp, c, cp = _csr(row_ptr, col)
    out = (ctypes.c_uint64 * 3)()
    rc = _load().oracle_count(len(rp) - 1, rpp, cp, int(k), int(nthreads), out)
    if rc != 0:
        raise ValueError("oracle_count rejected the input (rc=%d)" % rc)
    return int(out[0]) | (int(out[1]) << 64), int(out[2])


def count_roots(row_ptr, col, k: int, roots, nthreads: int = 0):
    """Per-root (count, fp) for the k-cliques whose minimum vertex under the
    (degree, id) order is each given root."""
    rp, rpp, c, cp = _csr(row_ptr, col)
    r, rptr = _i32(roots if len(roots) else np.zeros(1, np.int32))
    nr = len(roots)
    out = np.zeros(3 * max(nr, 1), dtype=np.uint64)
    rc = _load().oracle_count_roots(
        len(rp) - 1, rpp, cp, int(k), rptr, nr, int(nthreads),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise ValueError("oracle_count_roots rejected the input (rc=%d)" % rc)
    res = []
    for i in range(nr):
        res.append((int(out[3 * i]) | (int(out[3 * i + 1]) << 64),
                    int(out[3 * i + 2])))
    return res


def pivot_count_roots(row_ptr, col, k: int, roots, nthreads: int = 0):
    """The same per-root (count, fp) as count_roots, by pivoting (secondary
    reference for dense neighbourhoods; k <= 16)."""
    rp, rpp, c, cp = _csr(row_ptr, col)
    r, rptr = _i32(roots if len(roots) else np.zeros(1, np.int32))
    nr = len(roots)
    out = np.zeros(3 * max(nr, 1), dtype=np.uint64)
    rc = _load().oracle_pivot_count_roots(
        len(rp) - 1, rpp, cp, int(k), rptr, nr, int(nthreads),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise ValueError("oracle_pivot_count_roots rejected the input (rc=%d)" % rc)
    res = []
    for i in range(nr):
        res.append((int(out[3 * i]) | (int(out[3 * i + 1]) << 64),
                    int(out[3 * i + 2])))
    return res


def list_cliques(row_ptr, col, k: int, cap: int = 1 << 24) -> np.ndarray:
    """All k-cliques as an (N, k) int32 array of input ids, each row sorted,
    rows in lexicographic order."""
    rp, rpp, c, cp = _csr(row_ptr, col)
    lib = _load()
    total = lib.oracle_list(len(rp) - 1, rpp, cp, int(k), None, 0)
    if total < 0:
        raise ValueError("oracle_list rejected the input")
    if total > cap:
        raise ValueError("%d cliques exceed cap %d" % (total, cap))
    out = np.zeros((max(total, 1), k), dtype=np.int32)
    got = lib.oracle_list(len(rp) - 1, rpp, cp, int(k),
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          total)
    assert got == total
    return out[:total]


def soft_embed(dag_ptr, dag_col) -> np.ndarray:
    """Algorithm 5 on a DAG whose order is the vertex index order."""
    p, pp = _i32(dag_ptr)
    c, cp = _i32(dag_col if len(dag_col) else np.zeros(1, np.int32))
    n = len(p) - 1
    r = np.zeros(max(n, 1), dtype=np.int32)
    rc = _load().oracle_soft_embed(n, pp, cp,
                                   r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc != 0:
        raise ValueError("not a DAG in index order")
    return r[:n]


def root_soft_embed(row_ptr, col) -> np.ndarray:
    """r_{G'}(u), G' = G[N+(u) u {u}], under the (degree, id) order."""
    rp, rpp, c, cp = _csr(row_ptr, col)
    n = len(rp) - 1
    r = np.zeros(max(n, 1), dtype=np.int32)
    rc = _load().oracle_root_soft_embed(
        n, rpp, cp, r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc != 0:
        raise ValueError("oracle_root_soft_embed rejected the input")
    return r[:n]


def degeneracy(row_ptr, col):
    """(degeneracy, removal order) by minimum-degree removal, ties to the
    smallest id."""
    rp, rpp, c, cp = _csr(row_ptr, col)
    n = len(rp) - 1
    order = np.zeros(max(n, 1), dtype=np.int32)
    d = _load().oracle_degeneracy(
        n, rpp, cp, order.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if d < 0:
        raise ValueError("oracle_degeneracy failed")
    return int(d), order[:n]


def degree_rank(row_ptr) -> np.ndarray:
    rp, rpp = _i32(row_ptr)
    n = len(rp) - 1
    rank = np.zeros(max(n, 1), dtype=np.int32)
    rc = _load().oracle_degree_rank(
        n, rpp, rank.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc != 0:
        raise ValueError("oracle_degree_rank failed")
    return rank[:n]
