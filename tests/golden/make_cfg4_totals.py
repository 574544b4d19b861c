"""Writes cfg4_totals.json: the (count, fingerprint) of every pair of the
batched workload (4,096 Chung-Lu graphs, n ~ U{50..5000}, exponent ~
U[2.1, 3.0], mean degree ~ U[4, 40], 0-3 planted cliques of 8..25 vertices,
each paired with k ~ U{3..12}; seed 4), computed on the CPU by the oracle
only: the pivot-based counter over every root of each graph, summed (each
clique is counted once, at its minimum vertex).  The file holds the SHA-256
of the per-pair list "count,fp" (one line per pair, in pair order), the sums,
and the first 256 pairs verbatim.

Run from the repository root: python tests/golden/make_cfg4_totals.py"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

P61 = (1 << 61) - 1


def pair_digest(results):
    """SHA-256 of the per-pair list, one "count,fp" line per pair."""
    text = "".join("%d,%d\n" % (c, f) for c, f in results)
    return hashlib.sha256(text.encode()).hexdigest()


def main():
    import numpy as np
    import oracle
    from paper_2502_00317_amd import graphgen as gg
    t = time.time()
    specs = gg.batch_specs()
    graphs = gg.batch_graphs(specs)
    results = []
    for s, g in zip(specs, graphs):
        per = oracle.pivot_count_roots(g.row_ptr, g.col, s["k"], np.arange(g.n, dtype=np.int32))
        results.append((sum(c for c, _ in per), sum(f for _, f in per) % P61))
    out = {"workload": "4,096 Chung-Lu graphs n~U{50..5000}, exponent~U[2.1,3.0], mean degree~U[4,40], "
                       "0-3 planted cliques of 8..25, k~U{3..12}, seed 4",
           "pairs": len(results), "edges": int(sum(g.m for g in graphs)),
           "sha256": pair_digest(results),
           "sum_count": str(sum(c for c, _ in results)),
           "sum_fp": str(sum(f for _, f in results) % P61),
           "first": [[str(c), str(f)] for c, f in results[:256]],
           "source": "oracle.pivot_count_roots over every root of each graph",
           "cpu_s": round(time.time() - t, 1)}
    with open(os.path.join(HERE, "cfg4_totals.json"), "w") as f:
        json.dump(out, f, indent=0)
    print({k: v for k, v in out.items() if k != "first"})


if __name__ == "__main__":
    main()
