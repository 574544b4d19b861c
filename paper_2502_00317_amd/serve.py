"""Continuous-batching query server for k-clique counts.

A pool of oriented graphs stays resident on the device.  Queries (graph, k)
arrive at any time -- against a pool graph, or with an ad-hoc graph uploaded
with the query.  S slots run batches concurrently, each on its own HIP
stream: whenever a slot is free it takes every admissible queued query and
counts them all in one dist_count_batch call, so queries that arrive while
other batches are on the GPU start as soon as a slot is free, and batches of
different slots overlap on the device.

Admission is memory-gated: an ad-hoc graph needs device memory for its
oriented form (estimated from n and m); it is admitted only while the
resident pool plus the admitted ad-hoc graphs fit the memory limit, and its
memory is released when its query completes.  Pool queries need no memory
and are never held back by an ad-hoc query that does not fit.

Each query carries a time budget; a query whose search exceeds it is
stopped on the device (the other queries of its batch go on) and reported
as DNF.  Latency is completion time minus arrival time.

The device work goes through a backend object, so the scheduling logic can
be exercised on the CPU with a simulated device (tests/fake_device.py).
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np


def oriented_bytes(n: int, m: int) -> int:
    """Device bytes of an oriented graph: rank, orig, dptr, roots, root
    degrees (5 x 4n), fingerprint weights (8n) and out-lists (4m), plus the
    transient input copy and scratch of orientation (about 12(n + 2m))."""
    return 28 * n + 4 * m + 12 * (n + 2 * m) + (1 << 20)


@dataclass
class Query:
    qid: int
    k: int
    t_arrival: float                 # seconds after the server start
    graph: int | None = None         # pool graph id
    adhoc: tuple | None = None       # (row_ptr, col) uploaded with the query
    deadline_ms: int = 0
    # filled in by the server
    count: int | None = None
    fp: int | None = None
    status: str = "pending"          # ok | overflow | dnf | error
    t_start: float | None = None
    t_done: float | None = None
    slot: int | None = None
    batch_size: int = 0
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def latency(self):
        return None if self.t_done is None else self.t_done - self.t_arrival

    def need_bytes(self) -> int:
        if self.adhoc is None:
            return 0
        rp, col = self.adhoc
        return oriented_bytes(len(rp) - 1, len(col) // 2)


class DeviceBackend:
    """The real device: dist (libdist.so) with one torch stream per slot."""

    def __init__(self, slots: int, cfg_kwargs=None):
        import torch
        from . import dist
        self.dist = dist
        self.torch = torch
        torch.cuda.init()
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.cfg = dist.config(**(cfg_kwargs or {}))

    def orient(self, row_ptr, col, slot):
        return self.dist.orient(row_ptr, col, stream=self.streams[slot])

    def free(self, g):
        g.free()

    def count_batch(self, slot, graphs, ks, deadlines_ms):
        res, rc, ms, st = self.dist.count_batch(graphs, ks, cfg=self.cfg, use_graph=False,
                                                stream=self.streams[slot],
                                                deadlines_ms=deadlines_ms, with_status=True)
        D = self.dist
        names = {D.OK: "ok", D.E_OVERFLOW: "overflow", D.E_CANCELLED: "dnf"}
        return res, [names.get(s, "error") for s in st], ms


class Server:
    def __init__(self, backend, pool_handles: dict, slots: int = 2,
                 mem_limit: int = 1 << 62, pool_bytes: int = 0, max_batch: int = 4096,
                 clock=time.perf_counter):
        self.pool_bytes = pool_bytes
        self.backend = backend
        self.pool = pool_handles
        self.slots = slots
        self.mem_limit = mem_limit
        self.mem_used = pool_bytes
        self.peak_mem = pool_bytes
        self.max_batch = max_batch
        self.clock = clock
        self.t0 = None
        self.pending = collections.deque()
        self.cv = threading.Condition()
        self.stopping = False
        self.threads = []
        self.batches = []     # (slot, size, t_start, t_end, device ms)
        self.errors = []

    # ---- lifecycle ------------------------------------------------------------
    def start(self):
        self.t0 = self.clock()
        for s in range(self.slots):
            t = threading.Thread(target=self._slot_loop, args=(s,), daemon=True)
            t.start()
            self.threads.append(t)

    def now(self):
        return self.clock() - self.t0

    def submit(self, q: Query):
        with self.cv:
            self.pending.append(q)
            self.cv.notify_all()
        return q

    def stop(self):
        with self.cv:
            self.stopping = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()

    # ---- scheduling -----------------------------------------------------------
    def _take(self):
        """Every admissible pending query, in arrival order, up to
        max_batch.  Called with the lock held."""
        taken = []
        keep = collections.deque()
        while self.pending and len(taken) < self.max_batch:
            q = self.pending.popleft()
            need = q.need_bytes()
            if need > self.mem_limit - self.pool_bytes:
                # can never fit, even with nothing else admitted
                q.status = "rejected"
                q.t_done = self.now()
                q.done.set()
                continue
            if need and self.mem_used + need > self.mem_limit:
                keep.append(q)  # waits for memory; pool queries may pass it
                continue
            self.mem_used += need
            self.peak_mem = max(self.peak_mem, self.mem_used)
            taken.append(q)
        keep.extend(self.pending)
        self.pending = keep
        return taken

    def _slot_loop(self, slot):
        while True:
            with self.cv:
                batch = self._take()
                while not batch:
                    if self.stopping and not self.pending:
                        return
                    self.cv.wait(0.05)
                    batch = self._take()
            self._run(slot, batch)

    def _run(self, slot, batch):
        t_start = self.now()
        adhoc = []
        graphs = []
        try:
            for q in batch:
                q.t_start = t_start
                q.slot = slot
                q.batch_size = len(batch)
                if q.adhoc is not None:
                    g = self.backend.orient(q.adhoc[0], q.adhoc[1], slot)
                    adhoc.append(g)
                    graphs.append(g)
                else:
                    graphs.append(self.pool[q.graph])
            res, status, ms = self.backend.count_batch(slot, graphs, [q.k for q in batch],
                                                       [q.deadline_ms for q in batch])
        except Exception as e:  # reported per query; the server keeps running
            self.errors.append(repr(e))
            res = [(None, None)] * len(batch)
            status = ["error"] * len(batch)
            ms = 0.0
        for g in adhoc:
            self.backend.free(g)
        t_end = self.now()
        with self.cv:
            for q, (c, f), st in zip(batch, res, status):
                q.count, q.fp, q.status = c, f, st
                q.t_done = t_end
                self.mem_used -= q.need_bytes()
                q.done.set()
            self.batches.append((slot, len(batch), t_start, t_end, ms))
            self.cv.notify_all()


def replay(server: Server, queries, sleep=time.sleep, log=None):
    """Open-loop load: submit every query at its arrival time (seconds after
    the server start) and wait for all of them.  Latency counts from the
    scheduled arrival, so a late submission is charged to the server."""
    order = sorted(queries, key=lambda q: q.t_arrival)
    for i, q in enumerate(order):
        delay = q.t_arrival - server.now()
        if delay > 0:
            sleep(delay)
        server.submit(q)
        if log and (i + 1) % 500 == 0:
            log("serving: %d/%d submitted at t=%.2f s" % (i + 1, len(order), server.now()))
    for q in order:
        q.done.wait()


def summarize(queries, wall_s: float):
    done = [q for q in queries if q.status in ("ok", "overflow")]
    lat = np.array([q.latency for q in done]) if done else np.zeros(1)
    cliques = sum(q.count for q in done)
    return {
        "queries": len(queries),
        "completed": len(done),
        "dnf": sum(q.status == "dnf" for q in queries),
        "rejected": sum(q.status == "rejected" for q in queries),
        "errors": sum(q.status == "error" for q in queries),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "max_ms": float(lat.max() * 1e3),
        "cliques": cliques,
        "cliques_per_s": cliques / wall_s if wall_s > 0 else 0.0,
        "qps": len(done) / wall_s if wall_s > 0 else 0.0,
        "wall_s": wall_s,
    }
