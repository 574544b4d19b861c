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

Within a batch, queries are scheduled cheapest first (by the predicted
search size) and each one is completed as soon as the device has finished
it, not when its whole batch ends; each slot's launches take a share of the
device's wavefront slots so that the batches of all slots run side by side.

Each query carries a latency budget counted from its arrival.  When its
batch is dispatched, what is left of the budget becomes its device budget;
a query whose search runs past it is stopped on the device (the other
queries of its batch go on) and reported as DNF, and a query whose budget
ran out while it waited is reported as DNF without running.  Latency is
completion time minus arrival time.

The device work goes through a backend object, so the scheduling logic can
be exercised on the CPU with a simulated device (tests/fake_device.py).
"""
from __future__ import annotations

import collections
import math
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
    deadline_ms: int = 0             # latency budget from arrival; 0 = none
    # filled in by the server
    count: int | None = None
    fp: int | None = None
    status: str = "pending"          # ok | overflow | dnf | error
    t_start: float | None = None
    t_done: float | None = None
    slot: int | None = None
    batch_size: int = 0
    lane: str = ""                   # express | bulk
    moves: int = 0                   # times moved from the express to the bulk lane
    handle: object = None            # oriented ad-hoc graph while the query lives
    owner: int = 0                   # batch that holds the query now
    admitted: bool = False           # its memory is counted
    est: float | None = None         # cost estimate used for routing
    released: bool = False
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

    def __init__(self, slots: int, cfg_kwargs=None, grid_pcts=None, slot_cfgs=None):
        """grid_pcts[s]: share of the device's wavefront slots that the
        launches of slot s may take (default: an equal share each), so that
        the batches of all slots are resident together; slot_cfgs[s]: further
        switches for slot s."""
        import torch
        from . import dist
        self.dist = dist
        self.torch = torch
        torch.cuda.init()
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        if grid_pcts is None:
            grid_pcts = [max(1, 100 // slots)] * slots
        slot_cfgs = slot_cfgs or [{}] * slots
        self.cfgs = [dist.config(**dict(cfg_kwargs or {}, grid_pct=int(p), **sc))
                     for p, sc in zip(grid_pcts, slot_cfgs)]
        self.cfg_one = dist.config(**dict(cfg_kwargs or {}))

    def estimate(self, g, k):
        return self.dist.estimate_cost(g, k)

    def orient(self, row_ptr, col, slot):
        return self.dist.orient(row_ptr, col, stream=self.streams[slot])

    def free(self, g):
        g.free()

    def count_batch(self, slot, graphs, ks, deadlines_ms, on_done=None, costs=None):
        """Counts every pair; on_done(i, count, fp, status, device_ms) is
        called for each pair as soon as it is finished on the device; pairs
        run in ascending order of costs."""
        D = self.dist
        names = {D.OK: "ok", D.E_OVERFLOW: "overflow", D.E_CANCELLED: "dnf"}
        cb = None
        if on_done is not None:
            def cb(i, c, f, st, dms):
                on_done(i, c, f, names.get(st, "error"), dms)
        t = time.perf_counter()
        if cb is None:
            res, rc, ms, st = D.count_batch(graphs, ks, cfg=self.cfgs[slot], use_graph=False,
                                            stream=self.streams[slot],
                                            deadlines_ms=deadlines_ms, with_status=True)
        else:
            res, rc, st = D.count_batch_stream(graphs, ks, cb, cfg=self.cfgs[slot],
                                               stream=self.streams[slot],
                                               deadlines_ms=deadlines_ms, costs=costs)
            ms = (time.perf_counter() - t) * 1e3
        return res, [names.get(s, "error") for s in st], ms

    def count_all(self, slot, g, kmax, budget_ms):
        """Every clique size k <= kmax of one graph in one pivot-based pass
        (dist_count_all), with the whole device: ([(count, fp)] per k,
        status)."""
        import ctypes
        D = self.dist
        cfg = D.Config()
        ctypes.memmove(ctypes.byref(cfg), ctypes.byref(self.cfg_one), ctypes.sizeof(cfg))
        cfg.deadline_ms = int(budget_ms)
        try:
            res, rc = D.count_all(g, int(kmax), cfg=cfg, stream=self.streams[slot])
        except D.DistError:
            return None, "error"
        if rc == D.E_CANCELLED:
            return None, "dnf"
        return res, "ok"

    def count_one(self, slot, g, k, budget_ms):
        """The per-graph call (dist_count_ex) for one query, with the whole
        device."""
        import ctypes
        D = self.dist
        cfg = D.Config()
        ctypes.memmove(ctypes.byref(cfg), ctypes.byref(self.cfg_one), ctypes.sizeof(cfg))
        cfg.deadline_ms = int(budget_ms)
        try:
            c, f, rc = D.count(g, k, cfg=cfg, stream=self.streams[slot])
        except D.DistError as e:
            return (None, None), ("dnf" if e.status == D.E_CANCELLED else "error")
        return (c, f), ("overflow" if rc == D.E_OVERFLOW else "ok")


class Server:
    """Continuous-batching server.

    slots      -- concurrent batches (one host thread and one stream each);
    express_ms -- when > 0 and slots >= 2, slot 0 is an express lane: its
                  batches give every query at most express_ms of device time;
                  a query cut off there moves to the bulk lane (the other
                  slots) with what is left of its latency budget, and later
                  queries with the same (pool graph, k) go to the bulk lane
                  directly.  This is a two-level feedback queue: light
                  queries never wait behind heavy ones;
    express_batch_ms -- an express batch takes queries, cheapest predicted
                  first, while their predicted device times add up to at most
                  this (a query never seen counts as express_ms), so an
                  express batch stays short;
    shed_frac  -- a (graph, k) that ran for at least shed_frac of the latency
                  budget in the bulk lane and was cut off is reported DNF at
                  once when it arrives again, without using the device; so is
                  a new query whose estimate is at least the smallest such
                  cut-off's for its k (unless a query with at least that
                  estimate has completed in the bulk lane);
    plain      -- one query at a time through the per-graph call (the
                  baseline without batching);
    stream_results -- complete each query as soon as the device reports it,
                  not when its whole batch ends;
    pivot_k    -- with pivot_k > 0, the bulk lane answers its pool queries of
                  k >= pivot_k by pivot-based counting, one pass per graph for
                  every k it holds (dist_count_all under the longest remaining
                  budget of those queries); a graph whose pass runs out of
                  budget goes back to the search for good, and its queries
                  return to the bulk queue with what is left of their budgets;
    router_table -- routing state to start from (router_state() of an
                  earlier run): the per-k thresholds of both lanes, the
                  (graph, k) known to be heavy or hopeless, and measured
                  service times;
    learn      -- update that state from this run's completions (False: the
                  table is frozen, so routing, shedding and batch order
                  depend only on the arrival stream, and p50/p99 repeat from
                  the seed up to device timing).
    """

    def __init__(self, backend, pool_handles: dict, slots: int = 2,
                 mem_limit: int = 1 << 62, pool_bytes: int = 0, max_batch: int = 4096,
                 clock=time.perf_counter, stream_results: bool = True, express_ms: int = 0,
                 plain: bool = False, express_batch_ms: float = 0.0, shed_frac: float = 0.0,
                 router_table: dict | None = None, learn: bool = True, pivot_k: int = 0):
        self.stream_results = stream_results
        self.pool_bytes = pool_bytes
        self.backend = backend
        self.pool = pool_handles
        self.slots = slots
        self.mem_limit = mem_limit
        self.mem_used = pool_bytes
        self.peak_mem = pool_bytes
        self.max_batch = 1 if plain else max_batch
        self.plain = plain
        self.clock = clock
        self.express_ms = express_ms if (express_ms > 0 and slots >= 2 and not plain) else 0
        self.express_batch_ms = express_batch_ms if express_batch_ms > 0 else 4.0 * self.express_ms
        self.shed_frac = shed_frac
        self.bulk_cut_ms = {}  # (pool graph, k) -> longest device time before a bulk cut-off
        self.bulk_heavy_min = {}  # k -> smallest estimate cut off in the bulk lane (hopeless)
        self.bulk_light_max = {}  # k -> largest estimate completed in the bulk lane
        self.shed = 0
        self.lanes = (["express"] + ["bulk"] * (slots - 1)) if self.express_ms else ["bulk"] * slots
        self.t0 = None
        self.queues = {"express": collections.deque(), "bulk": collections.deque()}
        self.heavy = set()    # (pool graph, k) cut off in the express lane
        self.service_ms = {}  # (pool graph, k) -> last measured device service time
        self.light_max = {}   # k -> largest estimate completed in the express lane
        self.heavy_min = {}   # k -> smallest estimate cut off in the express lane
        self.routed_bulk = 0  # queries sent to the bulk lane on arrival
        self.demoted = 0
        self.cv = threading.Condition()
        self.stopping = False
        self.threads = []
        self.batches = []     # (slot, size, t_start, t_end, device ms, t_count_start)
        self.errors = []
        self._batch_ids = 0
        self._running = {}    # slot -> batch id while a batch runs
        self.learn = learn
        self.pivot_k = pivot_k if (pivot_k > 0 and not plain) else 0
        self.pivot_slow = set()   # pool graphs whose pivot pass ran out of budget
        self.pivot_passes = 0
        if router_table:
            self.load_router(router_table)

    # ---- routing state ----------------------------------------------------------
    def router_state(self) -> dict:
        """The routing state as JSON-serialisable data (see load_router)."""
        def per_k(d):
            return {str(k): v for k, v in sorted(d.items()) if math.isfinite(v)}

        def per_pair(d):
            return [[int(g), int(k), float(v)] for (g, k), v in sorted(d.items())]

        return {"light_max": per_k(self.light_max), "heavy_min": per_k(self.heavy_min),
                "bulk_light_max": per_k(self.bulk_light_max), "bulk_heavy_min": per_k(self.bulk_heavy_min),
                "heavy": [[int(g), int(k)] for g, k in sorted(self.heavy)],
                "bulk_cut_ms": per_pair(self.bulk_cut_ms), "service_ms": per_pair(self.service_ms)}

    def load_router(self, t: dict):
        self.light_max = {int(k): float(v) for k, v in t.get("light_max", {}).items()}
        self.heavy_min = {int(k): float(v) for k, v in t.get("heavy_min", {}).items()}
        self.bulk_light_max = {int(k): float(v) for k, v in t.get("bulk_light_max", {}).items()}
        self.bulk_heavy_min = {int(k): float(v) for k, v in t.get("bulk_heavy_min", {}).items()}
        self.heavy = {(int(g), int(k)) for g, k in t.get("heavy", [])}
        self.bulk_cut_ms = {(int(g), int(k)): float(v) for g, k, v in t.get("bulk_cut_ms", [])}
        self.service_ms = {(int(g), int(k)): float(v) for g, k, v in t.get("service_ms", [])}

    # ---- lifecycle ------------------------------------------------------------
    def start(self):
        self.t0 = self.clock()
        for s in range(self.slots):
            t = threading.Thread(target=self._slot_loop, args=(s,), daemon=True)
            t.start()
            self.threads.append(t)

    def now(self):
        return self.clock() - self.t0

    def _estimate(self, q):
        """The library's cost bound for a pool query, with the clique size
        capped at 5 (sum over roots of C(d+, min(k - 1, 4))): it orders the
        light queries well, and its scale is learned per k (see _route)."""
        if q.adhoc is not None or not hasattr(self.backend, "estimate"):
            return None
        if q.est is None:
            q.est = self.backend.estimate(self.pool[q.graph], min(q.k, 5))
        return q.est

    def _hopeless(self, q):
        """Known or predicted to need more than its budget.  Lock held."""
        if not self.shed_frac or q.adhoc is not None or not q.deadline_ms:
            return False
        key = (q.graph, q.k)
        if key in self.bulk_cut_ms:
            return self.bulk_cut_ms[key] >= self.shed_frac * q.deadline_ms
        est, hmin = q.est, self.bulk_heavy_min.get(q.k)
        return est is not None and hmin is not None and est >= hmin and est > self.bulk_light_max.get(q.k, -1.0)

    def _route(self, q):
        """express or bulk.  A (graph, k) cut off in the express lane before
        goes to the bulk lane.  Otherwise a monotone threshold per k: the
        smallest estimate cut off in the express lane so far, unless a query
        with at least that estimate has completed there.  Lock held."""
        if not self.express_ms:
            return "bulk"
        if q.adhoc is not None:
            return "express"
        if (q.graph, q.k) in self.heavy:
            return "bulk"
        est = self._estimate(q)
        hmin = self.heavy_min.get(q.k)
        if est is not None and hmin is not None and est >= hmin and est > self.light_max.get(q.k, -1.0):
            return "bulk"
        return "express"

    def submit(self, q: Query):
        if self.express_ms and q.adhoc is None:
            self._estimate(q)  # outside the lock: a library call
        with self.cv:
            if self._hopeless(q):
                q.lane = "shed"
                self.shed += 1
                self._complete(q, None, None, "dnf", self.now())
                self.cv.notify_all()
                return q
            q.lane = self._route(q)
            if q.lane == "bulk" and self.express_ms:
                self.routed_bulk += 1
            self.queues[q.lane].append(q)
            self.cv.notify_all()
        return q

    def stop(self):
        with self.cv:
            self.stopping = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()

    # ---- scheduling -----------------------------------------------------------
    def _idle(self):
        return not self.queues["express"] and not self.queues["bulk"]

    def _take(self, lane):
        """Every admissible pending query of the lane, in arrival order, up
        to max_batch.  Called with the lock held."""
        taken = []
        keep = collections.deque()
        pending = self.queues[lane]
        budget = None
        if lane == "express" and self.express_ms:
            # cheapest predicted first, while the predictions fit the batch budget
            pending = collections.deque(sorted(pending, key=self._predict_ms))
            budget = self.express_batch_ms
        while pending and len(taken) < self.max_batch:
            q = pending.popleft()
            if budget is not None:
                c = self._predict_ms(q)
                if taken and c > budget:
                    keep.append(q)
                    continue
                budget -= c
            if q.admitted:  # moved here from the express lane; memory held
                taken.append(q)
                continue
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
            q.admitted = True
            taken.append(q)
        keep.extend(pending)
        self.queues[lane] = keep
        return taken

    def _slot_loop(self, slot):
        lane = self.lanes[slot]
        while True:
            with self.cv:
                batch = self._take(lane)
                while not batch:
                    if self.stopping and self._idle() and not self._in_flight():
                        self.cv.notify_all()
                        return
                    self.cv.wait(0.05)
                    batch = self._take(lane)
                self._batch_ids += 1
                bid = self._batch_ids
                for q in batch:
                    q.owner = bid
                self._running[slot] = bid
            self._run(slot, lane, bid, batch)

    def _in_flight(self):
        # a running batch of the express lane may still move queries to the bulk lane
        return any(b is not None for b in self._running.values())

    def _complete(self, q, count, fp, status, t):
        """Called with the lock held."""
        if q.done.is_set():
            return
        q.count, q.fp, q.status = count, fp, status
        q.t_done = t
        q.done.set()

    def _settle(self, lane, q, res, status, cut, t, dms=-1.0):
        """A reported pair: complete it, or move it to the bulk lane when the
        express lane's budget (not its own) cut it off.  Lock held."""
        if self.learn:
            self._learn(lane, q, status, cut, dms)
        if status == "dnf" and lane == "express" and cut:
            q.lane = "bulk"
            q.moves += 1
            self.demoted += 1
            self.queues["bulk"].append(q)
            self.cv.notify_all()
            return
        self._complete(q, res[0], res[1], status, t)

    def _learn(self, lane, q, status, cut, dms):
        """Routing state from a reported pair.  Lock held."""
        if q.adhoc is None and status in ("ok", "overflow") and dms >= 0:
            self.service_ms[(q.graph, q.k)] = dms
        if q.adhoc is None and lane == "bulk" and status == "dnf" and dms >= 0:
            key = (q.graph, q.k)
            self.bulk_cut_ms[key] = max(self.bulk_cut_ms.get(key, 0.0), dms)
            if q.est is not None and q.deadline_ms and dms >= self.shed_frac * q.deadline_ms:
                self.bulk_heavy_min[q.k] = min(self.bulk_heavy_min.get(q.k, float("inf")), q.est)
        if q.adhoc is None and lane == "bulk" and status in ("ok", "overflow") and q.est is not None:
            self.bulk_light_max[q.k] = max(self.bulk_light_max.get(q.k, -1.0), q.est)
        if lane == "express" and q.est is not None:
            if status in ("ok", "overflow"):
                self.light_max[q.k] = max(self.light_max.get(q.k, -1.0), q.est)
            elif status == "dnf" and cut:
                self.heavy_min[q.k] = min(self.heavy_min.get(q.k, float("inf")), q.est)
        if status == "dnf" and lane == "express" and cut and q.adhoc is None:
            self.heavy.add((q.graph, q.k))

    def _predict_ms(self, q):
        ms = self.service_ms.get((q.graph, q.k)) if q.adhoc is None else None
        return ms if ms is not None else float(self.express_ms)

    def _costs(self, live, graphs):
        """Scheduling order of a batch: pairs measured before by their last
        service time, then the others by the library's cost bound."""
        out = []
        for q, g in zip(live, graphs):
            ms = self.service_ms.get((q.graph, q.k)) if q.adhoc is None else None
            if ms is not None:
                out.append(ms)
            else:
                est = self.backend.estimate(g, min(q.k, 5)) if hasattr(self.backend, "estimate") else 0.0
                out.append(1e9 + math.log10(1.0 + est))
        return out

    def _release(self, bid, batch):
        """Frees the ad-hoc graphs of finished queries this batch owns."""
        for q in batch:
            if q.done.is_set() and q.owner == bid and not q.released:
                q.released = True
                if q.handle is not None:
                    self.backend.free(q.handle)
                    q.handle = None
                with self.cv:
                    if q.admitted:
                        self.mem_used -= q.need_bytes()

    def _run(self, slot, lane, bid, batch):
        t_start = self.now()
        # queries whose latency budget ran out in the queue are not run
        with self.cv:
            for q in batch:
                if q.deadline_ms and (t_start - q.t_arrival) * 1e3 >= q.deadline_ms:
                    q.t_start = q.t_start if q.t_start is not None else t_start
                    q.slot = slot
                    self._complete(q, None, None, "dnf", t_start)
            self.cv.notify_all()
        live = [q for q in batch if not q.done.is_set()]
        if lane == "bulk" and self.pivot_k and hasattr(self.backend, "count_all"):
            passes = self.pivot_passes
            live = self._pivot_pass(slot, live, t_start)
            if self.pivot_passes != passes:
                t_start = self.now()  # the rest's budgets run from here
        budgets, cut = [], []
        for q in live:
            rem = int(q.deadline_ms - (t_start - q.t_arrival) * 1e3) if q.deadline_ms else 0
            rem = max(1, rem) if q.deadline_ms else 0
            if lane == "express" and (rem == 0 or self.express_ms < rem):
                budgets.append(self.express_ms)
                cut.append(True)
            else:
                budgets.append(rem)
                cut.append(False)
        reported = [False] * len(live)
        ms = 0.0
        t_dev = t_start
        if live:
            try:
                graphs = []
                for q in live:
                    if q.t_start is None:
                        q.t_start = t_start
                    q.slot = slot
                    q.batch_size = len(live)
                    if q.adhoc is not None:
                        if q.handle is None:
                            q.handle = self.backend.orient(q.adhoc[0], q.adhoc[1], slot)
                        graphs.append(q.handle)
                    else:
                        graphs.append(self.pool[q.graph])
                ks = [q.k for q in live]
                t_dev = self.now()
                if self.plain:
                    res, status = [], []
                    for g, k, b in zip(graphs, ks, budgets):
                        r, st = self.backend.count_one(slot, g, k, b)
                        res.append(r)
                        status.append(st)
                else:
                    on_done = None
                    if self.stream_results:
                        def on_done(i, count, fp, st, dms=-1.0):
                            t = self.now()
                            with self.cv:
                                reported[i] = True
                                self._settle(lane, live[i], (count, fp), st, cut[i], t, dms)
                    kw = {"on_done": on_done} if on_done is not None else {}
                    kw["costs"] = self._costs(live, graphs)
                    res, status, ms = self.backend.count_batch(slot, graphs, ks, budgets, **kw)
            except Exception as e:  # reported per query; the server keeps running
                self.errors.append(repr(e))
                res = [(None, None)] * len(live)
                status = ["error"] * len(live)
            t_end = self.now()
            with self.cv:
                for i, q in enumerate(live):
                    if not reported[i]:
                        self._settle(lane, q, res[i], status[i], cut[i], t_end)
        t_end = self.now()
        self._release(bid, batch)
        with self.cv:
            self.batches.append((slot, len(live), t_start, t_end, ms, t_dev))
            self._running[slot] = None
            self.cv.notify_all()

    def _pivot_pass(self, slot, live, t_start):
        """The bulk lane's pivot path: pool queries of k >= pivot_k, grouped by
        graph, each group answered by one all-k pass.  Returns the queries left
        for the search."""
        groups = {}
        rest = []
        for q in live:
            if q.adhoc is None and self.pivot_k <= q.k <= 16 and q.graph not in self.pivot_slow:
                groups.setdefault(q.graph, []).append(q)
            else:
                rest.append(q)
        for gi, qs in groups.items():
            now = self.now()
            timed = all(q.deadline_ms for q in qs)
            # the longest remaining budget of the group; none if a query has none
            budget = max(q.deadline_ms - (now - q.t_arrival) * 1e3 for q in qs) if timed else 0.0
            if timed and budget <= 1.0:
                rest.extend(qs)   # the search path completes them as DNF
                continue
            for q in qs:
                if q.t_start is None:
                    q.t_start = t_start
                q.slot = slot
                q.batch_size = len(qs)
            try:
                res, st = self.backend.count_all(slot, self.pool[gi], max(q.k for q in qs),
                                                 max(1, int(budget)) if timed else 0)
            except Exception as e:  # reported per query; the server keeps running
                self.errors.append(repr(e))
                res, st = None, "error"
            t = self.now()
            self.pivot_passes += 1
            with self.cv:
                if st == "ok":
                    for q in qs:
                        c, f = res[q.k]
                        late = q.deadline_ms and (t - q.t_arrival) * 1e3 > q.deadline_ms
                        self._complete(q, None if late else c, None if late else f,
                                       "dnf" if late else ("overflow" if c >> 64 else "ok"), t)
                else:
                    self.pivot_slow.add(gi)
                    rest.extend(qs)
                self.cv.notify_all()
        return rest


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
        while not q.done.wait(10.0):
            if log:
                log("serving: waiting, %d/%d done at t=%.1f s" % (
                    sum(x.done.is_set() for x in order), len(order), server.now()))


def summarize(queries, wall_s: float):
    """Latency over every query: a query that did not finish (DNF, shed on
    arrival, rejected or failed) counts at its latency budget, a lower bound
    of what it would have taken, so shedding load cannot improve p50/p99.
    The completed-only figures and the DNF and shed counts stand beside them."""
    done = [q for q in queries if q.status in ("ok", "overflow")]
    lat_done = np.array([q.latency for q in done]) if done else np.zeros(1)

    def charged(q):
        if q.status in ("ok", "overflow"):
            return q.latency
        return (q.deadline_ms or 0) / 1e3 if q.deadline_ms else float("inf")

    lat_all = np.array([charged(q) for q in queries]) if queries else np.zeros(1)
    cliques = sum(q.count for q in done)
    n = max(len(queries), 1)
    dnf = sum(q.status == "dnf" for q in queries)
    return {
        "queries": len(queries),
        "completed": len(done),
        "dnf": dnf,
        "dnf_rate": dnf / n,
        "shed": sum(q.lane == "shed" for q in queries),
        "rejected": sum(q.status == "rejected" for q in queries),
        "errors": sum(q.status == "error" for q in queries),
        "p50_ms": float(np.percentile(lat_all, 50) * 1e3),
        "p99_ms": float(np.percentile(lat_all, 99) * 1e3),
        "latency_of_unfinished": "its budget (deadline_ms)",
        "p50_completed_ms": float(np.percentile(lat_done, 50) * 1e3),
        "p99_completed_ms": float(np.percentile(lat_done, 99) * 1e3),
        "max_completed_ms": float(lat_done.max() * 1e3),
        "cliques": cliques,
        "cliques_per_s": cliques / wall_s if wall_s > 0 else 0.0,
        "qps": len(done) / wall_s if wall_s > 0 else 0.0,
        "wall_s": wall_s,
    }
