"""Autotuner for batched counting.

Picks, per size bucket of a batch, the switches of dist_count_batch_ex that
run fastest on the device:

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
before it trusts a timing.  Results are stored in a JSON file keyed by the
bucket of the batch: log2 of the total number of edges and the largest k.
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
