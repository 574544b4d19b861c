"""Writes cfg2_totals.json: the k-clique count (128-bit) and fingerprint of
the one-large-graph workload (Chung-Lu n = 1,000,000, exponent 2.2, mean
degree 20, degrees capped at 5,000, plus 200 planted 30-cliques, seed 2) at
k = 5, 7 and 9, computed on the CPU by the oracle only:

  * every k: the pivot-based counter (oracle_pivot_count_roots) over all
    vertices as roots, summed -- each clique is counted at its minimum vertex
    under the (degree, id) order, so the per-root results add up to the total;
  * k = 5 also by the enumerating oracle (oracle_count), which must agree.

Run from the repository root: python tests/golden/make_cfg2_totals.py
(about an hour on 8 cores)."""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

P61 = (1 << 61) - 1


def main():
    import numpy as np
    import oracle
    from paper_2502_00317_amd import graphgen as gg
    ks = [int(x) for x in (sys.argv[1] if len(sys.argv) > 1 else "5,7,9").split(",")]
    g = gg.large_powerlaw()
    roots = np.arange(g.n, dtype=np.int32)
    out = {"graph": "Chung-Lu n=1,000,000, exponent 2.2, mean degree 20, cap 5000, +200 planted K30, seed 2",
           "n": g.n, "m": g.m, "results": {}}
    path = os.path.join(HERE, "cfg2_totals.json")
    if os.path.exists(path):
        with open(path) as f:
            old = json.load(f)
        if old.get("n") == g.n and old.get("m") == g.m:
            out["results"] = old.get("results", {})
    for k in ks:
        t = time.time()
        per = oracle.pivot_count_roots(g.row_ptr, g.col, k, roots)
        count = sum(c for c, _ in per)
        fp = sum(f for _, f in per) % P61
        rec = {"count": str(count), "fp": str(fp), "source": "oracle.pivot_count_roots over all roots",
               "cpu_s": round(time.time() - t, 1)}
        if k == 5:
            t = time.time()
            c2, f2 = oracle.count(g.row_ptr, g.col, k)
            assert (c2, f2) == (count, fp), ("enumeration and pivoting disagree", c2, f2, count, fp)
            rec["source"] += "; equal to oracle.count (enumeration)"
            rec["enum_cpu_s"] = round(time.time() - t, 1)
        out["results"][str(k)] = rec
        print(k, rec, flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
