"""Autotuner for batched counting.

Picks, per size bucket of a batch, the switches of dist_count_batch_ex /
dist_count_batch_tuned that run fastest on the device:

* ``min_width``  -- smallest bitmap width (words of 64 bits, one of the
  library's width classes) given to a root; larger values merge the small
  width classes into fewer, wider launches (fewer tails, more LDS per wave);
* ``chunk_work`` -- work-unit size for roots with more than 64
  out-neighbours (children per unit = chunk_work / d; 0 = the library's
  cost-based sizing): smaller values split heavy roots across more
  wavefronts;
* ``memo``       -- memoisation of dense branches on or off.

Every candidate must return exactly the same (count, fingerprint) for every
pair -- the switches never change a result -- and the tuner checks that
before it trusts a timing.

Two granularities:

* ``tune_batch`` -- one set of switches for the whole batch, stored under
  the batch's bucket (log2 of the total number of edges and the largest k);
* ``tune_buckets`` -- the pairs are bucketed by the width class of their
  graph's largest out-degree (the bitmap width, 64..1024 bits, and with it
  the LDS a root takes) and by a band of k (how deep the search goes); each
  bucket's pairs are timed alone under every candidate, and the whole batch
  then runs once with each pair given its bucket's winner
  (dist_count_batch_tuned: still one launch per width class).  Winners are
  stored per bucket key, so a later batch with pairs of the same buckets
  reuses them without timing.
"""
from __future__ import annotations

import json
import math
import os
import time

DEFAULT_CANDIDATES = [
    dict(min_width=1, chunk_work=512, memo=1),
    dict(min_width=2, chunk_work=512, memo=1),
    dict(min_width=1, chunk_work=128, memo=1),
    dict(min_width=1, chunk_work=512, memo=0),
    dict(min_width=1, chunk_work=0, memo=1),
]


def bucket_key(total_edges: int, kmax: int) -> str:
    return "m2^%d/k%d" % (int(math.log2(max(total_edges, 1))), kmax)


class TuningDB:
    def __init__(self, path: str | None = None):
        self.path = path
        self.table = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.table = json.load(f)

    def get(self, key):
        return self.table.get(key)

    def put(self, key, entry):
        self.table[key] = entry
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.table, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def tune_batch(dist, graphs, ks, total_edges: int, db: TuningDB | None = None,
               candidates=None, reps: int = 1, fingerprint: int = 1, log=None):
    """Time every candidate on this batch (after one warm-up run each),
    check that all agree, store and return (best switches, report)."""
    candidates = candidates or DEFAULT_CANDIDATES
    key = bucket_key(total_edges, max(ks) if ks else 0)
    report = []
    ref = None
    best = None
    for cand in candidates:
        # a candidate slower than 3x the best so far is cut off by a deadline
        limit = int(max(2000.0, 3.0 * best[1])) if best else 0
        cfg = dist.config(fingerprint=fingerprint, deadline_ms=limit, **cand)
        res, rc, _ = dist.count_batch(graphs, ks, cfg=cfg, use_graph=True)  # plan + warm-up
        if rc == dist.E_CANCELLED:
            report.append(dict(cand, ms=None, note="over %d ms" % limit))
            if log:
                log("autotune %s: cut off at %d ms" % (cand, limit))
            continue
        if ref is None:
            ref = res
        if res != ref:
            raise RuntimeError("autotune: candidate %r changed a result" % (cand,))
        times = []
        for _ in range(reps):
            t = time.perf_counter()
            r2, rc, ms = dist.count_batch(graphs, ks, cfg=cfg, use_graph=True)
            times.append((time.perf_counter() - t) * 1e3)
            if r2 != ref:
                raise RuntimeError("autotune: replay of %r changed a result" % (cand,))
        ms_best = min(times)
        report.append(dict(cand, ms=ms_best))
        if log:
            log("autotune %s: %.1f ms" % (cand, ms_best))
        if best is None or ms_best < best[1]:
            best = (cand, ms_best)
    if db is not None:
        db.put(key, {"switches": best[0], "ms": best[1], "candidates": report})
    return best[0], report


WIDTHS = (1, 2, 3, 4, 5, 6, 8, 16)
K_BANDS = ((1, 5), (6, 8), (9, 12), (13, 64))


def width_class(max_outdeg: int) -> int:
    """Words per bitmap row of the library's width class for this out-degree."""
    need = max(1, (int(max_outdeg) + 63) // 64)
    for w in WIDTHS:
        if w >= need:
            return w
    return WIDTHS[-1]


def k_band(k: int) -> int:
    for i, (lo, hi) in enumerate(K_BANDS):
        if lo <= k <= hi:
            return i
    return len(K_BANDS) - 1


def pair_bucket(max_outdeg: int, k: int) -> str:
    lo, hi = K_BANDS[k_band(k)]
    return "w%d/k%d-%d" % (width_class(max_outdeg), lo, hi)


def bucket_pairs(max_outdegs, ks):
    """{bucket key: [pair indices]} in first-appearance order."""
    out = {}
    for i, (d, k) in enumerate(zip(max_outdegs, ks)):
        out.setdefault(pair_bucket(d, k), []).append(i)
    return out


def _time_candidate(dist, graphs, ks, cfg, reps):
    res, rc, _ = dist.count_batch(graphs, ks, cfg=cfg, use_graph=True)  # plan + warm-up
    if rc == dist.E_CANCELLED:
        return res, rc, None
    times = []
    for _ in range(reps):
        t = time.perf_counter()
        r2, rc2, _ = dist.count_batch(graphs, ks, cfg=cfg, use_graph=True)
        times.append((time.perf_counter() - t) * 1e3)
        if r2 != res:
            raise RuntimeError("autotune: a replay changed a result")
    return res, rc, min(times)


def tune_buckets(dist, graphs, ks, db: TuningDB | None = None, candidates=None, reps: int = 2,
                 fingerprint: int = 1, log=None, retune: bool = False):
    """Per-bucket switches for a batch: returns (per-pair switch dicts,
    {bucket: entry}).  A bucket already in db is not timed again unless
    retune is set.  Every candidate of a bucket must give the same results."""
    candidates = candidates or DEFAULT_CANDIDATES
    degs = [g.info().max_outdeg for g in graphs]
    buckets = bucket_pairs(degs, ks)
    chosen = {}
    for key, idx in buckets.items():
        entry = db.get(key) if (db is not None and not retune) else None
        if entry is None:
            sub_g = [graphs[i] for i in idx]
            sub_k = [ks[i] for i in idx]
            ref, best, report = None, None, []
            for cand in candidates:
                limit = int(max(2000.0, 3.0 * best[1])) if best else 0
                cfg = dist.config(fingerprint=fingerprint, deadline_ms=limit, **cand)
                res, rc, ms = _time_candidate(dist, sub_g, sub_k, cfg, reps)
                if ms is None:
                    report.append(dict(cand, ms=None, note="over %d ms" % limit))
                    continue
                if ref is None:
                    ref = res
                if res != ref:
                    raise RuntimeError("autotune: candidate %r changed a result in %s" % (cand, key))
                report.append(dict(cand, ms=ms))
                if best is None or ms < best[1]:
                    best = (cand, ms)
            entry = {"switches": best[0], "ms": best[1], "pairs": len(idx), "candidates": report}
            if db is not None:
                db.put(key, entry)
            if log:
                log("autotune %s (%d pairs): %s in %.1f ms" % (key, len(idx), best[0], best[1]))
        chosen[key] = entry
    per_pair = [None] * len(ks)
    for key, idx in buckets.items():
        for i in idx:
            per_pair[i] = dict(chosen[key]["switches"])
    return per_pair, chosen
