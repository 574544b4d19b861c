"""Thin ctypes binding of libdist.so (include/dist.h).

Argument marshalling only: every step of orientation and search runs in the
HIP kernels of the library.  The library is loaded on first use; if it has
not been built this raises instead of falling back to anything else.

Arrays may be NumPy arrays (host) or torch tensors (host or device); device
tensors are passed as raw device pointers, and the HIP stream is taken from
``torch.cuda.current_stream()`` when torch has a device.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdist.so")

OK, E_INVALID, E_K, E_NOMEM, E_DEVICE, E_OVERFLOW, E_CANCELLED, E_UNSUPPORTED, E_SCRATCH = range(9)
WIDTHS = (1, 2, 3, 4, 5, 6, 8, 16)   # DIST_WIDTHS: bitmap width classes (words)
WIDTH_CLASSES = len(WIDTHS)
ORDER_DEGREE, ORDER_DEGENERACY, ORDER_INPUT = 0, 1, 2
K_MAX = 64
P61 = (1 << 61) - 1


class DistError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what, strerror(status) if _lib else "", status))


class Config(ctypes.Structure):
    _fields_ = [("memo", ctypes.c_int32), ("prune", ctypes.c_int32),
                ("fingerprint", ctypes.c_int32), ("memo_entries", ctypes.c_int32),
                ("memo_bytes", ctypes.c_int64), ("deadline_ms", ctypes.c_int64),
                ("chunk_work", ctypes.c_int32), ("grid_pct", ctypes.c_int32),
                ("budget_from_pair_start", ctypes.c_int32), ("min_width", ctypes.c_int32),
                ("sub_units", ctypes.c_int32), ("trie_nodes", ctypes.c_int32),
                ("list_bytes", ctypes.c_int64), ("trie_tau", ctypes.c_int64),
                ("edge_units", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("count_lo", ctypes.c_uint64), ("count_hi", ctypes.c_uint64),
                ("fp", ctypes.c_uint64)]

    @property
    def count(self) -> int:
        return int(self.count_lo) | (int(self.count_hi) << 64)


class PairSwitches(ctypes.Structure):
    """dist_pair_switches: per-pair min_width, chunk_work, memo (< 0: the
    batch's; min_width 0 also)."""
    _fields_ = [("min_width", ctypes.c_int32), ("chunk_work", ctypes.c_int32),
                ("memo", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("roots", ctypes.c_uint64), ("roots_pruned", ctypes.c_uint64),
                ("frames", ctypes.c_uint64), ("word_ops", ctypes.c_uint64),
                ("leaf_bits", ctypes.c_uint64), ("memo_lookups", ctypes.c_uint64),
                ("memo_hits", ctypes.c_uint64), ("memo_inserts", ctypes.c_uint64),
                ("subgraph_arcs", ctypes.c_uint64), ("kernel_ms", ctypes.c_double),
                ("bucket_ms", ctypes.c_double * WIDTH_CLASSES), ("bucket_roots", ctypes.c_uint64 * WIDTH_CLASSES),
                ("bucket_word_ops", ctypes.c_uint64 * WIDTH_CLASSES),
                ("bucket_leaf_bits", ctypes.c_uint64 * WIDTH_CLASSES),
                ("bucket_arcs", ctypes.c_uint64 * WIDTH_CLASSES)]

    def as_dict(self):
        out = {}
        for f, _ in self._fields_:
            v = getattr(self, f)
            out[f] = list(v) if hasattr(v, "__len__") else v
        return out


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64), ("order_mode", ctypes.c_int32),
                ("max_outdeg", ctypes.c_int32), ("order_bound", ctypes.c_int32),
                ("orient_ms", ctypes.c_double)]


PAIR_DONE = ctypes.CFUNCTYPE(None, ctypes.c_int, ctypes.POINTER(Result), ctypes.c_int,
                             ctypes.c_double, ctypes.c_void_p)

SINK = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.c_uint64,
                        ctypes.c_int, ctypes.c_void_p)

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdist.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2502_00317_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.dist_config_init.argtypes = [ctypes.POINTER(Config)]
    lib.dist_config_init.restype = None
    lib.dist_strerror.argtypes = [ctypes.c_int]
    lib.dist_strerror.restype = ctypes.c_char_p
    lib.dist_orient.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int,
                                ctypes.POINTER(Config), vp, ctypes.POINTER(vp)]
    lib.dist_orient.restype = ctypes.c_int
    lib.dist_count.argtypes = [vp, ctypes.c_int, vp, ctypes.POINTER(Result)]
    lib.dist_count.restype = ctypes.c_int
    lib.dist_count_ex.argtypes = [vp, ctypes.c_int, ctypes.POINTER(Config), vp, vp,
                                  ctypes.POINTER(Result)]
    lib.dist_count_ex.restype = ctypes.c_int
    lib.dist_count_noalloc.argtypes = [vp, ctypes.c_int, ctypes.POINTER(Config), vp, ctypes.POINTER(Result)]
    lib.dist_count_noalloc.restype = ctypes.c_int
    lib.dist_list.argtypes = [vp, ctypes.c_int, SINK, vp, vp, ctypes.POINTER(Result)]
    lib.dist_list.restype = ctypes.c_int
    lib.dist_count_all.argtypes = [vp, ctypes.c_int, ctypes.POINTER(Config), vp, ctypes.c_int, vp,
                                   ctypes.POINTER(Result)]
    lib.dist_count_all.restype = ctypes.c_int
    lib.dist_list_ex.argtypes = [vp, ctypes.c_int, ctypes.POINTER(Config), ctypes.c_int, SINK, vp, vp,
                                 ctypes.POINTER(Result)]
    lib.dist_list_ex.restype = ctypes.c_int
    lib.dist_ist_inspect.argtypes = [vp, ctypes.c_int, ctypes.c_int32, ctypes.POINTER(Config), vp, ctypes.c_int,
                                     ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_int32), vp, vp, vp, vp,
                                     ctypes.POINTER(ctypes.c_int32), vp, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), vp]
    lib.dist_ist_inspect.restype = ctypes.c_int
    lib.dist_count_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int),
                                     ctypes.c_int, vp, ctypes.POINTER(Result)]
    lib.dist_count_batch.restype = ctypes.c_int
    lib.dist_count_batch_ex.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int),
                                        ctypes.c_int, ctypes.POINTER(Config), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int64), vp,
                                        ctypes.POINTER(Result), ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_double)]
    lib.dist_count_batch_ex.restype = ctypes.c_int
    lib.dist_count_batch_tuned.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int),
                                           ctypes.c_int, ctypes.POINTER(Config), ctypes.POINTER(PairSwitches),
                                           ctypes.c_int, ctypes.POINTER(ctypes.c_int64), vp,
                                           ctypes.POINTER(Result), ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_double)]
    lib.dist_count_batch_tuned.restype = ctypes.c_int
    lib.dist_count_batch_stream.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int),
                                            ctypes.c_int, ctypes.POINTER(Config),
                                            ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_double), vp,
                                            ctypes.POINTER(Result), ctypes.POINTER(ctypes.c_int),
                                            PAIR_DONE, vp]
    lib.dist_count_batch_stream.restype = ctypes.c_int
    lib.dist_estimate_cost.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.dist_estimate_cost.restype = ctypes.c_int
    lib.dist_mem_cached.argtypes = [ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.dist_mem_cached.restype = ctypes.c_int
    lib.dist_mem_trim.argtypes = []
    lib.dist_mem_trim.restype = ctypes.c_int
    lib.dist_root_soft_embed.argtypes = [vp, ctypes.c_int, vp, vp]
    lib.dist_root_soft_embed.restype = ctypes.c_int
    lib.dist_graph_ranks.argtypes = [vp, vp, vp]
    lib.dist_graph_ranks.restype = ctypes.c_int
    lib.dist_graph_info_get.argtypes = [vp, ctypes.POINTER(GraphInfo)]
    lib.dist_graph_info_get.restype = ctypes.c_int
    lib.dist_stats_get.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.dist_stats_get.restype = ctypes.c_int
    lib.dist_graph_free.argtypes = [vp]
    lib.dist_graph_free.restype = None
    _lib = lib
    return lib


def lib():
    return _load()


def strerror(status: int) -> str:
    return _load().dist_strerror(int(status)).decode()


def config(**kw) -> Config:
    c = Config()
    _load().dist_config_init(ctypes.byref(c))
    for k, v in kw.items():
        if not hasattr(c, k):
            raise TypeError("unknown config field %r" % k)
        setattr(c, k, v)
    return c


def _stream_ptr(stream):
    if stream is not None:
        return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    try:
        import torch
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return ctypes.c_void_p(0)


def _ptr(a, dtype):
    """(pointer, keepalive) for a NumPy array or torch tensor."""
    if hasattr(a, "data_ptr"):  # torch tensor
        return ctypes.c_void_p(a.data_ptr()), a
    arr = np.ascontiguousarray(a, dtype=dtype)
    if arr.size == 0:
        arr = np.zeros(1, dtype=dtype)
    return ctypes.c_void_p(arr.ctypes.data), arr


class Graph:
    """An oriented graph resident on the device (owns a dist_graph*)."""

    def __init__(self, handle, n):
        self._h = handle
        self.n = n

    @property
    def handle(self):
        return self._h

    def __del__(self):
        self.free()

    def free(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dist_graph_free(self._h)
            self._h = None

    def info(self) -> GraphInfo:
        out = GraphInfo()
        _check(_load().dist_graph_info_get(self._h, ctypes.byref(out)), "dist_graph_info_get")
        return out

    def stats(self) -> Stats:
        out = Stats()
        _check(_load().dist_stats_get(self._h, ctypes.byref(out)), "dist_stats_get")
        return out

    def ranks(self, stream=None) -> np.ndarray:
        out = np.zeros(max(self.n, 1), np.int32)
        _check(_load().dist_graph_ranks(self._h, ctypes.c_void_p(out.ctypes.data),
                                        _stream_ptr(stream)), "dist_graph_ranks")
        return out[: self.n]


def _check(rc, what):
    if rc != OK:
        raise DistError(rc, what)


def orient(row_ptr, col, order=ORDER_DEGREE, cfg: Config | None = None, stream=None) -> Graph:
    """dist_orient on a CSR graph (NumPy or torch arrays)."""
    n = len(row_ptr) - 1
    nnz = len(col)
    rp, k1 = _ptr(row_ptr, np.int32)
    cp, k2 = _ptr(col, np.int32)
    h = ctypes.c_void_p()
    rc = _load().dist_orient(rp, cp, n, nnz, int(order),
                             ctypes.byref(cfg) if cfg is not None else None,
                             _stream_ptr(stream), ctypes.byref(h))
    _check(rc, "dist_orient")
    return Graph(h, n)


def count(g: Graph, k: int, cfg: Config | None = None, per_root=None, stream=None,
          allow_overflow=True):
    """(count as Python int, fp, status).  per_root: optional array of 3*n
    uint64 (NumPy host array or torch device tensor) filled per input id."""
    res = Result()
    if cfg is None and per_root is None:
        rc = _load().dist_count(g.handle, int(k), _stream_ptr(stream), ctypes.byref(res))
    else:
        pr = None
        keep = None
        if per_root is not None:
            pr, keep = _ptr(per_root, np.uint64)
        rc = _load().dist_count_ex(g.handle, int(k),
                                   ctypes.byref(cfg) if cfg is not None else None,
                                   pr, _stream_ptr(stream), ctypes.byref(res))
    if rc not in (OK, E_OVERFLOW) or (rc == E_OVERFLOW and not allow_overflow):
        _check(rc, "dist_count")
    return res.count, int(res.fp), rc


ALL_K_MAX = 16


def count_all(g: Graph, kmax: int, cfg: Config | None = None, per_root=None, per_root_k: int = 0, stream=None):
    """dist_count_all: [(count, fp) for k = 0 .. kmax] by pivoting, and the
    status.  per_root: optional 3*n uint64 (NumPy or torch device tensor),
    filled per input id for k = per_root_k."""
    out = (Result * (int(kmax) + 1))()
    pr, keep = (None, None)
    if per_root is not None:
        pr, keep = _ptr(per_root, np.uint64)
    rc = _load().dist_count_all(g.handle, int(kmax), ctypes.byref(cfg) if cfg is not None else None, pr,
                                int(per_root_k), _stream_ptr(stream), out)
    if rc not in (OK, E_OVERFLOW, E_CANCELLED):
        _check(rc, "dist_count_all")
    return [(r.count, int(r.fp)) for r in out], rc


def count_noalloc(g: Graph, k: int, cfg: Config | None = None, stream=None, allow_overflow=True):
    """dist_count_noalloc: (count, fp, status) without any device allocation
    (static scratch; no memo, no per-root output)."""
    res = Result()
    rc = _load().dist_count_noalloc(g.handle, int(k), ctypes.byref(cfg) if cfg is not None else None,
                                    _stream_ptr(stream), ctypes.byref(res))
    if rc not in (OK, E_OVERFLOW) or (rc == E_OVERFLOW and not allow_overflow):
        _check(rc, "dist_count_noalloc")
    return res.count, int(res.fp), rc


def count_batch(graphs, ks, cfg: Config | None = None, use_graph=True, stream=None,
                deadlines_ms=None, with_status=False):
    """dist_count_batch_ex: ([(count, fp)] per pair, status, device ms), plus
    the per-pair statuses when with_status is set."""
    n = len(graphs)
    arr = (ctypes.c_void_p * max(n, 1))(*[g.handle for g in graphs])
    karr = (ctypes.c_int * max(n, 1))(*[int(k) for k in ks])
    out = (Result * max(n, 1))()
    st = (ctypes.c_int * max(n, 1))()
    dl = None
    if deadlines_ms is not None:
        dl = (ctypes.c_int64 * max(n, 1))(*[int(x) for x in deadlines_ms])
    ms = ctypes.c_double(0)
    rc = _load().dist_count_batch_ex(arr, karr, n, ctypes.byref(cfg) if cfg is not None else None,
                                     1 if use_graph else 0, dl, _stream_ptr(stream), out, st,
                                     ctypes.byref(ms))
    if rc not in (OK, E_OVERFLOW, E_CANCELLED):
        _check(rc, "dist_count_batch")
    res = [(out[i].count, int(out[i].fp)) for i in range(n)]
    if with_status:
        return res, rc, ms.value, [int(st[i]) for i in range(n)]
    return res, rc, ms.value


def count_batch_tuned(graphs, ks, switches, cfg: Config | None = None, use_graph=True, stream=None,
                      deadlines_ms=None):
    """dist_count_batch_tuned: count_batch with per-pair switches; switches[i]
    is a dict with any of min_width, chunk_work, memo (missing: the batch's).
    Returns ([(count, fp)] per pair, status, device ms)."""
    n = len(graphs)
    arr = (ctypes.c_void_p * max(n, 1))(*[g.handle for g in graphs])
    karr = (ctypes.c_int * max(n, 1))(*[int(k) for k in ks])
    sw = (PairSwitches * max(n, 1))()
    for i, d in enumerate(switches):
        sw[i].min_width = int(d.get("min_width", 0))
        sw[i].chunk_work = int(d.get("chunk_work", -1))
        sw[i].memo = int(d.get("memo", -1))
    out = (Result * max(n, 1))()
    st = (ctypes.c_int * max(n, 1))()
    dl = None
    if deadlines_ms is not None:
        dl = (ctypes.c_int64 * max(n, 1))(*[int(x) for x in deadlines_ms])
    ms = ctypes.c_double(0)
    rc = _load().dist_count_batch_tuned(arr, karr, n, ctypes.byref(cfg) if cfg is not None else None, sw,
                                        1 if use_graph else 0, dl, _stream_ptr(stream), out, st, ctypes.byref(ms))
    if rc not in (OK, E_OVERFLOW, E_CANCELLED):
        _check(rc, "dist_count_batch_tuned")
    return [(out[i].count, int(out[i].fp)) for i in range(n)], rc, ms.value


def count_batch_stream(graphs, ks, on_done, cfg: Config | None = None, stream=None,
                       deadlines_ms=None, costs=None):
    """dist_count_batch_stream: on_done(i, count, fp, status, device_ms) is
    called for every pair as soon as the device has finished it; pairs are
    scheduled in ascending order of costs (None: the library's estimate).
    Returns ([(count, fp)] per pair, status, per-pair statuses)."""
    n = len(graphs)
    arr = (ctypes.c_void_p * max(n, 1))(*[g.handle for g in graphs])
    karr = (ctypes.c_int * max(n, 1))(*[int(k) for k in ks])
    out = (Result * max(n, 1))()
    st = (ctypes.c_int * max(n, 1))()
    dl = None
    if deadlines_ms is not None:
        dl = (ctypes.c_int64 * max(n, 1))(*[int(x) for x in deadlines_ms])
    cost = None
    if costs is not None:
        cost = (ctypes.c_double * max(n, 1))(*[float(x) for x in costs])
    errors = []

    def _cb(i, res, status, dms, user):
        try:
            r = res.contents
            on_done(int(i), r.count, int(r.fp), int(status), float(dms))
        except BaseException as e:  # never unwind through C
            errors.append(e)

    cb = PAIR_DONE(_cb)
    rc = _load().dist_count_batch_stream(arr, karr, n, ctypes.byref(cfg) if cfg is not None else None,
                                         dl, cost, _stream_ptr(stream), out, st, cb, None)
    if errors:
        raise errors[0]
    if rc not in (OK, E_OVERFLOW, E_CANCELLED):
        _check(rc, "dist_count_batch_stream")
    return [(out[i].count, int(out[i].fp)) for i in range(n)], rc, [int(st[i]) for i in range(n)]


def mem_cached():
    """(device bytes, pinned host bytes) held in the library's block cache."""
    d, h = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(_load().dist_mem_cached(ctypes.byref(d), ctypes.byref(h)), "dist_mem_cached")
    return d.value, h.value


def mem_trim():
    _check(_load().dist_mem_trim(), "dist_mem_trim")


def estimate_cost(g: Graph, k: int) -> float:
    v = ctypes.c_double(0)
    _check(_load().dist_estimate_cost(g.handle, int(k), ctypes.byref(v)), "dist_estimate_cost")
    return v.value


LIST_DEVICE_ROWS = 1


def list_cliques(g: Graph, k: int, sink=None, stream=None, cfg: Config | None = None, device_rows=False,
                 raw_sink=None):
    """dist_list / dist_list_ex.  With sink=None (and no raw_sink) returns
    (rows array (N, k) int32, count, fp, status); otherwise calls
    sink(np.ndarray (n, k)) per chunk, or raw_sink(ptr, n, k) with the
    library's pointer (a device pointer with device_rows), and returns
    (None, count, fp, status)."""
    chunks = []

    def _cb(ptr, n, kk, user):
        if raw_sink is not None:
            return int(bool(raw_sink(ctypes.cast(ptr, ctypes.c_void_p).value, int(n), kk)))
        arr = np.ctypeslib.as_array(ptr, shape=(int(n) * kk,)).reshape(int(n), kk).copy()
        if sink is None:
            chunks.append(arr)
            return 0
        return int(bool(sink(arr)))

    cb = SINK(_cb)
    res = Result()
    if cfg is None and not device_rows:
        rc = _load().dist_list(g.handle, int(k), cb, None, _stream_ptr(stream), ctypes.byref(res))
    else:
        rc = _load().dist_list_ex(g.handle, int(k), ctypes.byref(cfg) if cfg is not None else None,
                                  LIST_DEVICE_ROWS if device_rows else 0, cb, None, _stream_ptr(stream),
                                  ctypes.byref(res))
    if rc not in (OK, E_OVERFLOW, E_CANCELLED):
        _check(rc, "dist_list")
    rows = None
    if sink is None and raw_sink is None:
        rows = np.concatenate(chunks) if chunks else np.zeros((0, k), np.int32)
    return rows, res.count, int(res.fp), rc


def ist_inspect(g: Graph, k: int, root: int, cfg: Config | None = None, ret_set=None, ret_l: int = 0,
                cap: int = 1 << 14, rows_cap: int = 1 << 16, stream=None):
    """dist_ist_inspect: the Induced Subgraph Trie built while listing the
    k-cliques of one root, and one ListingIST retrieval.  Returns a dict with
    local_ids, nodes (list of frozensets of input ids; node 0 the root),
    marked (list of int bit masks), lc / ls (lists of per-l node ids), rows
    (the root's cliques) and retrieved (the retrieval's cliques)."""
    local = np.zeros(1024, np.int32)
    d = ctypes.c_int32(0)
    sets = np.zeros((cap + 1) * 16, np.uint64)
    marked = np.zeros(cap + 1, np.uint64)
    lc = np.zeros((cap + 1) * k, np.uint32)
    ls = np.zeros((cap + 1) * k, np.uint32)
    nn = ctypes.c_int32(0)
    rows = np.zeros(max(rows_cap, 1) * k, np.int32)
    nr = ctypes.c_int64(0)
    nret = ctypes.c_int64(0)
    rs = None
    if ret_set is not None:
        rs = np.zeros(16, np.uint64)
        rs[: len(ret_set)] = np.asarray(ret_set, np.uint64)
    rc = _load().dist_ist_inspect(
        g.handle, int(k), int(root), ctypes.byref(cfg) if cfg is not None else None,
        ctypes.c_void_p(rs.ctypes.data) if rs is not None else None, int(ret_l), int(cap),
        ctypes.c_void_p(local.ctypes.data), ctypes.byref(d), ctypes.c_void_p(sets.ctypes.data),
        ctypes.c_void_p(marked.ctypes.data), ctypes.c_void_p(lc.ctypes.data), ctypes.c_void_p(ls.ctypes.data),
        ctypes.byref(nn), ctypes.c_void_p(rows.ctypes.data), int(rows_cap), ctypes.byref(nr), ctypes.byref(nret),
        _stream_ptr(stream))
    _check(rc, "dist_ist_inspect")
    n = nn.value
    ids = local[: d.value]
    nodes = []
    for t in range(n):
        bits = sets[t * 16:(t + 1) * 16]
        mem = [int(ids[w * 64 + b]) for w in range(16) for b in range(64) if (int(bits[w]) >> b) & 1]
        nodes.append(frozenset(mem))
    r = rows[: (nr.value + nret.value) * k].reshape(-1, k)
    return {"local_ids": ids.copy(), "nodes": nodes, "marked": [int(m) for m in marked[:n]],
            "lc": lc[: n * k].reshape(n, k).copy(), "ls": ls[: n * k].reshape(n, k).copy(),
            "rows": r[: nr.value].copy(), "retrieved": r[nr.value:].copy()}


def root_soft_embed(g: Graph, cap: int, stream=None) -> np.ndarray:
    out = np.zeros(max(g.n, 1), np.int32)
    _check(_load().dist_root_soft_embed(g.handle, int(cap), ctypes.c_void_p(out.ctypes.data),
                                        _stream_ptr(stream)), "dist_root_soft_embed")
    return out[: g.n]
