#!/usr/bin/env python3
"""Benchmark: k-clique counting on one MI355X (plain per-graph path).

Workload: Chung-Lu graph, n = 1,000,000, power-law exponent 2.2, mean
degree 20, degrees capped at 5,000, plus 200 planted 30-cliques (seed 2;
synthetic stand-in for the paper's real networks).  One step = the whole
hot path on the resident CSR: dist_orient (degree order) followed by
dist_count for every k of --ks (default 5, 7 and 9), each with its count and
fingerprint.  Untimed legs beside it: pivot-based counting of every k in one
pass, listing on the Induced Subgraph Trie, the dense-core R-MAT graph under
a deadline, the batched workload and serving.

Prints one JSON line with the metric, the roofline of the dominant search
kernel (integer ALU bound) and the CPU oracle timed on a bounded sample of
the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 lanes x 2.4 GHz = 39.3e12 32-bit integer lane-ops/s
PEAK_INT_LANE_OPS = 256 * 64 * 2.4e9
# algorithmic lane-ops per unit of work:
OPS_PER_WORD_OP = 4    # 2 x v_and_b32 + 2 x v_bcnt_u32_b32 on one 64-bit word
OPS_PER_LEAF_BIT = 2   # one 64-bit add of a fingerprint weight
BUCKET_W = [1, 2, 3, 4, 5, 6, 8, 16]   # the library's width classes (DIST_WIDTHS)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ks", default="5,7,9")
    ap.add_argument("--fp-ks", default="all",
                    help="ks whose fingerprint is computed ('all' = every k of --ks; the rest: exact count only)")
    ap.add_argument("--k-dnf", type=int, default=0, help="a further k attempted once under a deadline")
    ap.add_argument("--dnf-deadline-ms", type=int, default=20000)
    ap.add_argument("--order", default="degree", choices=["degree", "degeneracy"])
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--cpu-stride", type=int, default=8, help="oracle sample: every s-th vertex as root")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain-equiv", action="store_true",
                    help="skip the per-root i-clique counts behind the plain-equivalent work figure "
                         "(--no-cpu skips them too)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched (4,096 graph) section")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving section")
    ap.add_argument("--serve-queries", type=int, default=2000)
    ap.add_argument("--serve-deadline-ms", type=int, default=2000)
    ap.add_argument("--serve-express-ms", type=int, default=50,
                    help="device budget of the express lane (0: no express lane)")
    ap.add_argument("--serve-trace", default="", help="write per-query and per-batch serving records here")
    ap.add_argument("--serve-bulk-slots", type=int, default=1)
    ap.add_argument("--serve-express-batch-ms", type=float, default=200.0,
                    help="predicted device time of one express batch")
    ap.add_argument("--serve-shed-frac", type=float, default=0.5,
                    help="report a (graph, k) DNF at once after a bulk cut-off that ran this share of the budget")
    ap.add_argument("--serve-modes", default="served,plain")
    ap.add_argument("--serve-pivot-k", type=int, default=6,
                    help="served mode: the bulk lane answers pool queries of k >= this by one pivot-based "
                         "all-k pass per graph (0 = off)")
    ap.add_argument("--state-dir", default="", metavar="DIR",
                    help="write the autotuner's database and, when the router learns online, its routing "
                         "state here (default: keep them in memory)")
    ap.add_argument("--serve-router", default=os.path.join(ROOT, "paper_2502_00317_amd", "router_cfg5.json"),
                    help="routing table of the served mode (stored from an earlier run's router_state); "
                         "used frozen when the file exists, else the router learns online")
    ap.add_argument("--serve-express-pct", type=int, default=45,
                    help="share of the device's wavefront slots for the express lane")
    ap.add_argument("--summarize-profiles", default="", metavar="DIR",
                    help="turn rocprofv3 CSVs under DIR into the summaries under profiles/")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device (calibrates rocprofv3 FETCH/WRITE_SIZE)")
    ap.add_argument("--no-listing", action="store_true", help="skip the listing section")
    ap.add_argument("--no-pivot", action="store_true", help="skip the pivot-based all-k section")
    ap.add_argument("--no-cfg3", action="store_true", help="skip the dense-core R-MAT attempt")
    ap.add_argument("--cfg3-deadline-ms", type=int, default=5000)
    ap.add_argument("--cfg3-k6-deadline-ms", type=int, default=200000,
                    help="deadline of the dense-core k=6 count (degree order); 0 skips it")
    ap.add_argument("--out", default="")
    return ap.parse_args()


KERNEL_SOURCES = ["paper_2502_00317_amd/csrc/search.hip", "paper_2502_00317_amd/csrc/device_common.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_search_cfg2_traffic.json")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def summarize_profiles(d):
    """Per-launch HBM traffic of the search kernels from two rocprofv3 --pmc
    runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the
    same counter reads for a 1 GiB device-to-device copy."""
    import csv
    import glob

    def rows(sub):
        f = glob.glob(os.path.join(d, sub, "*counter_collection.csv"))
        return list(csv.DictReader(open(f[0])))

    out = {"source_hash": kernel_source_hash(), "kernels": {}, "calibration": {}}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        cal = [float(r["Counter_Value"]) for r in rows("pmccal_" + c) if "copyBuffer" in r["Kernel_Name"]]
        factor = (1 << 20) / cal[0]  # KiB of a 1 GiB copy / counter reading
        out["calibration"][c] = {"copy_KiB": 1 << 20, "counter_KiB": cal[0], "factor": factor}
        for r in rows("pmc_" + c):
            name = r["Kernel_Name"]
            if "k_search<" not in name:
                continue
            kname = "k_search<%s>" % name.split("k_search<")[1].split(",")[0]
            e = out["kernels"].setdefault(kname, {"FETCH_SIZE": [], "WRITE_SIZE": []})
            e[c].append(float(r["Counter_Value"]) * 1024.0 * factor)
    for kname, e in out["kernels"].items():
        n = max(len(e["FETCH_SIZE"]), 1)
        e["launches"] = n
        e["bytes_per_launch"] = (sum(e["FETCH_SIZE"]) + sum(e["WRITE_SIZE"])) / n
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    lines = ["# HBM traffic of the search kernels (rocprofv3 --pmc), plain count on the",
             "# Chung-Lu n=1e6 workload, k = 5 (fingerprint), 7 and 9, one launch each",
             "",
             "Commands (repository root, one MI355X; TMPDIR=/tmp; OUT = an absolute results directory):",
             "",
             "    rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/pmc_FETCH_SIZE -o run -- \\",
             "        python3 $PWD/bench.py --steps 1 --warmup 0 --no-cpu --no-batched --no-serving --no-pivot --no-listing --no-cfg3",
             "    rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/pmc_WRITE_SIZE -o run -- \\",
             "        python3 $PWD/bench.py --steps 1 --warmup 0 --no-cpu --no-batched --no-serving --no-pivot --no-listing --no-cfg3",
             "    rocprofv3 --pmc FETCH_SIZE (and WRITE_SIZE) ... -- python3 $PWD/bench.py --calib-copy 1024",
             "    python3 bench.py --summarize-profiles $OUT",
             "",
             "Calibration (1 GiB device copy): FETCH_SIZE factor %.3f, WRITE_SIZE factor %.3f." % (
                 out["calibration"]["FETCH_SIZE"]["factor"], out["calibration"]["WRITE_SIZE"]["factor"]),
             "Kernel source hash: %s" % out["source_hash"],
             "",
             "| kernel | launches (k = 5, 7, 9) | fetched GB per launch | written GB per launch |",
             "|---|---|---|---|"]
    for kname, e in sorted(out["kernels"].items()):
        lines.append("| %s | %d | %s | %s |" % (kname, e["launches"],
                     " / ".join("%.2f" % (x / 1e9) for x in e["FETCH_SIZE"]),
                     " / ".join("%.2f" % (x / 1e9) for x in e["WRITE_SIZE"])))
    with open(os.path.join(ROOT, "profiles", "k_search_cfg2_traffic.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    stats = glob.glob(os.path.join(d, "prof", "*kernel_stats.csv"))
    if stats:
        lines = ["# rocprofv3 kernel summary: plain count, Chung-Lu n=1e6, k = 5 (fingerprint), 7 and 9",
                 "",
                 "Command (repository root, one MI355X; OUT = an absolute results directory):",
                 "",
                 "    export TMPDIR=/tmp",
                 "    rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/prof -o run -- \\",
                 "        python3 $PWD/bench.py --steps 1 --warmup 0 --no-cpu --no-batched --no-serving --no-pivot --no-listing --no-cfg3",
                 "    python3 bench.py --summarize-profiles $OUT",
                 "",
                 "One orientation (degree order) and one dist_count per k (one launch per width",
                 "class per k); k_search<W> is the search kernel for roots whose out-degree",
                 "needs W 64-bit words per bitmap row.  The average over the three launches is",
                 "the avg_launch_ms that bench.py reports for the dominant kernel.",
                 "Kernel source hash: %s" % out["source_hash"],
                 "",
                 "| kernel | calls | total ms | average ms | % |",
                 "|---|---|---|---|---|"]
        per_w = {}
        for r in csv.DictReader(open(stats[0])):
            name = r["Name"].replace("void (anonymous namespace)::", "").replace("((anonymous namespace)::Params)", "(Params)")
            lines.append("| %s | %s | %.3f | %.3f | %.2f |" % (name, r["Calls"], float(r["TotalDurationNs"]) / 1e6,
                                                           float(r["AverageNs"]) / 1e6, float(r["Percentage"])))
            if name.startswith("k_search<"):
                e = per_w.setdefault("k_search<%s>" % name.split("<")[1].split(",")[0], [0, 0.0])
                e[0] += int(r["Calls"])
                e[1] += float(r["TotalDurationNs"]) / 1e6
        lines += ["",
                  "Per width class, all instantiations together (the figure bench.py's",
                  "roofline.avg_launch_ms is compared with):",
                  "",
                  "| kernel | launches | total ms | average ms per launch |",
                  "|---|---|---|---|"]
        for kname, (n, ms) in sorted(per_w.items()):
            lines.append("| %s | %d | %.3f | %.3f |" % (kname, n, ms, ms / max(n, 1)))
        with open(os.path.join(ROOT, "profiles", "k_search_cfg2_kernel_stats.md"), "w") as f:
            f.write("\n".join(lines) + "\n")
    summarize_issue(d)
    legs = glob.glob(os.path.join(d, "prof_legs", "*kernel_stats.csv"))
    if legs:
        lines = ["# rocprofv3 kernel summary: one bench step plus its pivot-based all-k and listing",
                 "# sections (Chung-Lu n=1e6, k = 5, 7, 9; all k <= 9 by pivoting; listing on the",
                 "# Chung-Lu n=1e4 graph, k = 4 and 6)",
                 "",
                 "Command (repository root, one MI355X; OUT = an absolute results directory):",
                 "",
                 "    export TMPDIR=/tmp",
                 "    rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/prof_legs -o run -- \\",
                 "        python3 $PWD/bench.py --steps 1 --warmup 0 --no-cpu --no-batched --no-serving --no-cfg3",
                 "    python3 bench.py --summarize-profiles $OUT",
                 "",
                 "k_pivot<W> counts every clique size by pivoting (one launch per width class);",
                 "k_list_ist<W> lists cliques with the Induced Subgraph Trie (Algorithms 3 and 4).",
                 "Kernel sources hash (search.hip, device_common.h): %s" % out["source_hash"],
                 "",
                 "| kernel | calls | total ms | average ms | % |",
                 "|---|---|---|---|---|"]
        for r in csv.DictReader(open(legs[0])):
            name = r["Name"].replace("void (anonymous namespace)::", "").replace("(anonymous namespace)::", "")
            if float(r["Percentage"]) < 0.01:
                continue
            lines.append("| %s | %s | %.3f | %.3f | %.2f |" % (name, r["Calls"], float(r["TotalDurationNs"]) / 1e6,
                                                           float(r["AverageNs"]) / 1e6, float(r["Percentage"])))
        with open(os.path.join(ROOT, "profiles", "pivot_listing_kernel_stats.md"), "w") as f:
            f.write("\n".join(lines) + "\n")
    print(json.dumps(out)[:400])


def summarize_issue(d):
    """Instruction issue rates of the search kernels from two rocprofv3 --pmc
    runs of SQ counters (sq_1, sq_2 under d), against the issue peaks of
    256 CUs at 2.4 GHz: 4 SIMDs per CU, each issuing one wave64 VALU
    instruction per 4 cycles (614 G/s, the 39.3 T lane-op/s of the roofline),
    and one LDS instruction per CU per cycle (614 G/s)."""
    import csv
    import glob
    data = {}
    for sub in ("sq_1", "sq_2"):
        f = glob.glob(os.path.join(d, sub, "*counter_collection.csv"))
        if not f:
            return
        for r in csv.DictReader(open(f[0])):
            name = r["Kernel_Name"]
            if "k_search<" not in name:
                continue
            key = (int(r["Dispatch_Id"]), name.split("k_search<")[1].split(">")[0])
            e = data.setdefault((sub, key), {"ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
            e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    peak = 256 * 4 * 2.4e9 / 4
    lines = ["# Instruction issue of the search kernels (rocprofv3 --pmc SQ counters), plain count",
             "# on the Chung-Lu n=1e6 workload, k = 5 (fingerprint), 7 and 9",
             "",
             "Commands (repository root, one MI355X; TMPDIR=/tmp; OUT = an absolute results directory), one pass each:",
             "",
             "    rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_SMEM SQ_INSTS_BRANCH \\",
             "        SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR GRBM_GUI_ACTIVE --output-format csv -d $OUT/sq_1 -o run -- \\",
             "        python3 $PWD/bench.py --steps 1 --warmup 0 --no-cpu --no-batched --no-serving --no-pivot --no-listing --no-cfg3",
             "    rocprofv3 --pmc SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_LDS_BANK_CONFLICT SQ_BUSY_CYCLES SQ_WAVE_CYCLES \\",
             "        SQ_THREAD_CYCLES_VALU SQ_WAIT_INST_LDS SQ_ACTIVE_INST_ANY GRBM_COUNT --output-format csv \\",
             "        -d $OUT/sq_2 -o run -- python3 $PWD/bench.py --steps 1 --warmup 0 --no-cpu --no-batched --no-serving --no-pivot --no-listing --no-cfg3",
             "    python3 bench.py --summarize-profiles $OUT",
             "",
             "Peaks (256 CUs, 2.4 GHz): VALU 614 G wave64 instructions/s (4 SIMDs per CU, one wave64",
             "instruction per SIMD per 4 cycles = 39.3 T lane-ops/s); LDS 614 G instructions/s (one per CU",
             "per cycle).  k_search<W, EMIT, FP>: one launch per width class per k.",
             "Kernel source hash: %s" % kernel_source_hash(),
             "",
             "| kernel | k | ms | VALU G/s | VALU % of peak | SALU G/s | LDS G/s | LDS % of peak | bank-conflict cycles / LDS active cycles | VMEM rd+wr M |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    keys = sorted({k for (_, k) in data}, key=lambda x: (int(x[1].split(",")[0]), x[0]))
    nth = {}
    for key in keys:
        w = int(key[1].split(",")[0])
        kk = (5, 7, 9)[nth.get(w, 0)] if nth.get(w, 0) < 3 else "?"
        nth[w] = nth.get(w, 0) + 1
        a = data.get(("sq_1", key))
        b = data.get(("sq_2", key))
        if not a or not b:
            continue
        sec = a["ns"] / 1e9
        valu = a.get("SQ_INSTS_VALU", 0) / sec
        lds = a.get("SQ_INSTS_LDS", 0) / sec
        conf = b.get("SQ_LDS_BANK_CONFLICT", 0) / max(b.get("SQ_ACTIVE_INST_LDS", 1), 1)
        lines.append("| k_search<%s> | %s | %.1f | %.1f | %.1f | %.1f | %.1f | %.2f | %.2f | %.1f |" % (
            key[1], kk, a["ns"] / 1e6, valu / 1e9, 100 * valu / peak, a.get("SQ_INSTS_SALU", 0) / sec / 1e9,
            lds / 1e9, 100 * lds / peak, conf, (a.get("SQ_INSTS_VMEM_RD", 0) + a.get("SQ_INSTS_VMEM_WR", 0)) / 1e6))
    with open(os.path.join(ROOT, "profiles", "k_search_cfg2_issue.md"), "w") as f:
        f.write("\n".join(lines) + "\n")


def measured_traffic(kernel):
    """Calibrated bytes per launch of `kernel` from the committed counter
    summary, or None if the search kernel has changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    e = t["kernels"].get(kernel)
    return e["bytes_per_launch"] if e else None


def main():
    a = parse()
    if a.summarize_profiles:
        summarize_profiles(a.summarize_profiles)
        return
    if a.calib_copy:
        import torch
        n = a.calib_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": n}))
        return
    if a.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); the per-root work "
              "would shard across GPUs as described in DESIGN.md", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    from paper_2502_00317_amd import graphgen as gg

    # inputs of the batched section are generated in worker processes before
    # this process touches the GPU
    batch_specs = batch_graphs = None
    if not a.no_batched:
        t0 = time.time()
        batch_specs = gg.batch_specs(count=a.batch_count)
        batch_graphs = gg.batch_graphs(batch_specs)
        print("[bench] batched inputs: %d graphs, %d edges, %.1f s" % (
            len(batch_graphs), sum(g.m for g in batch_graphs), time.time() - t0), file=sys.stderr, flush=True)
    serve_inputs = None
    if not a.no_serving:
        t0 = time.time()
        pool_specs = gg.serving_pool_specs()
        queries = gg.serving_queries(count=a.serve_queries)
        adhoc_specs = [q["adhoc"] for q in queries if "adhoc" in q]
        graphs = gg.spec_graphs(pool_specs + adhoc_specs)
        serve_inputs = (pool_specs, queries, graphs[:len(pool_specs)], graphs[len(pool_specs):])
        print("[bench] serving inputs: pool %d graphs (%d edges), %d ad-hoc graphs, %.1f s" % (
            len(pool_specs), sum(g.m for g in graphs[:len(pool_specs)]), len(adhoc_specs), time.time() - t0),
            file=sys.stderr, flush=True)

    import torch
    from paper_2502_00317_amd import dist

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.init()
    dist.lib()
    ks = [int(x) for x in a.ks.split(",") if x]
    fp_ks = set(ks) if a.fp_ks == "all" else {int(x) for x in a.fp_ks.split(",") if x}
    order = dist.ORDER_DEGREE if a.order == "degree" else dist.ORDER_DEGENERACY

    t0 = time.time()
    g = gg.large_powerlaw(n=a.n)
    gen_s = time.time() - t0
    rp = torch.from_numpy(g.row_ptr).cuda()
    col = torch.from_numpy(g.col).cuda()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    cfgs = {k: dist.config(fingerprint=1 if k in fp_ks else 0) for k in ks}

    def log(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    log("graph n=%d m=%d generated in %.1f s" % (g.n, g.m, gen_s))

    per_k = {k: {"ms": [], "kernel_ms": [], "stats": None} for k in ks}
    results = {}
    orient_ms = []

    def step(record):
        t = time.perf_counter()
        G = dist.orient(rp, col, order=order, stream=stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if record:
            orient_ms.append((t1 - t) * 1e3)
        for k in ks:
            tk = time.perf_counter()
            cnt, fp, rc = dist.count(G, k, cfg=cfgs[k], stream=stream)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - tk) * 1e3
            log("k=%d count=%d fp=%d %.1f ms%s" % (k, cnt, fp, dt, "" if record else " (warmup)"))
            if rc not in (dist.OK, dist.E_OVERFLOW):
                raise RuntimeError("count failed k=%d rc=%d" % (k, rc))
            if k in results:
                assert results[k] == (cnt, fp), "nondeterministic result"
            results[k] = (cnt, fp)
            if record:
                st = G.stats()
                per_k[k]["ms"].append(dt)
                per_k[k]["kernel_ms"].append(st.kernel_ms)
                per_k[k]["stats"] = st.as_dict()
        return G

    for _ in range(a.warmup):
        step(False).free()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    G = None
    for _ in range(a.steps):
        if G is not None:
            G.free()
        G = step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / a.steps
    total_cliques = sum(results[k][0] for k in ks)
    value = total_cliques / (ms_per_step / 1e3)

    # ---- roofline of the dominant search kernel (bucket with most time) ----
    agg = {w: {"ms": 0.0, "wops": 0, "bits": 0, "launches": 0} for w in BUCKET_W}
    for k in ks:
        st = per_k[k]["stats"]
        for i, w in enumerate(BUCKET_W):
            if st["bucket_ms"][i] > 0:
                agg[w]["ms"] += st["bucket_ms"][i]
                agg[w]["wops"] += st["bucket_word_ops"][i]
                agg[w]["bits"] += st["bucket_leaf_bits"][i]
                agg[w]["launches"] += 1
    wdom = max(BUCKET_W, key=lambda w: agg[w]["ms"])
    A = agg[wdom]
    avg_launch_ms = A["ms"] / max(A["launches"], 1)
    ops_per_launch = (OPS_PER_WORD_OP * A["wops"] + OPS_PER_LEAF_BIT * A["bits"]) / max(A["launches"], 1)
    achieved = ops_per_launch / (avg_launch_ms / 1e3) / 1e12
    peak = PEAK_INT_LANE_OPS / 1e12
    roofline = {"bound": "alu", "kernel": "k_search<%d>" % wdom, "achieved": round(achieved, 4),
                "peak": round(peak, 2), "unit": "Tlane-op/s", "frac": round(achieved / peak, 5),
                "traffic": measured_traffic("k_search<%d>" % wdom), "avg_launch_ms": round(avg_launch_ms, 3),
                "ops_per_launch": ops_per_launch}

    # ---- k attempted under a deadline (not timed) ----
    dnf = None
    if a.k_dnf and a.k_dnf not in ks:
        log("k=%d under a %d ms deadline" % (a.k_dnf, a.dnf_deadline_ms))
        c2 = dist.config(deadline_ms=a.dnf_deadline_ms, fingerprint=0)
        try:
            cnt, fp, rc = dist.count(G, a.k_dnf, cfg=c2, stream=stream)
        except dist.DistError as e:
            cnt, fp, rc = None, None, e.status
        st = G.stats()
        dnf = {"k": a.k_dnf, "deadline_ms": a.dnf_deadline_ms,
               "status": "finished" if rc in (dist.OK, dist.E_OVERFLOW) else "DNF",
               "count": cnt, "fp": fp, "roots_done": st.roots, "kernel_ms": st.kernel_ms}

    # ---- plain-equivalent work (not timed) ----
    # A plain depth-first search over the same bitmaps computes one candidate
    # bitmap of W(u) words per i-clique rooted at u, i = 2..k-1; counting all
    # of them (4 lane-ops per word) overestimates the plain work slightly,
    # since the plain search skips children whose candidates are too few.
    if not (a.no_plain_equiv or a.no_cpu):
        rank = G.ranks(stream=stream).astype(np.int64)
        deg = np.diff(g.row_ptr).astype(np.int64)
        src = np.repeat(np.arange(g.n, dtype=np.int64), deg)
        outd = np.bincount(src[rank[src] < rank[g.col]], minlength=g.n)
        wid = np.zeros(g.n, np.float64)
        for w in reversed(BUCKET_W):
            wid[outd <= 64 * w] = w
        ci = {2: outd.astype(np.float64)}
        per = torch.zeros(3 * g.n, dtype=torch.int64, device="cuda")
        for i in range(3, max(ks)):
            per.zero_()
            dist.count(G, i, cfg=dist.config(fingerprint=0), per_root=per, stream=stream)
            torch.cuda.synchronize()
            h = per.cpu().numpy().view(np.uint64)
            ci[i] = h[0::3].astype(np.float64) + h[1::3].astype(np.float64) * 2.0 ** 64
        pe_ops = 0.0
        pe_ms = 0.0
        for k in ks:
            searched = outd >= k - 1
            pe_ops += OPS_PER_WORD_OP * float(np.sum(wid[searched] * sum(ci[i][searched] for i in range(2, k))))
            pe_ms += float(np.median(per_k[k]["kernel_ms"]))
        rate = pe_ops / (pe_ms / 1e3) / 1e12
        roofline["plain_equiv"] = {"lane_ops": pe_ops, "search_ms": round(pe_ms, 3), "rate": round(rate, 2),
                                   "unit": "Tlane-op/s", "x_peak": round(rate / peak, 2)}
        log("plain-equivalent work: %.3g lane-ops in %.0f ms of search, %.3g T lane-op/s (%.1fx the VALU peak)" % (
            pe_ops, pe_ms, rate, rate / peak))

    # ---- sampled parity at full size: per-root results vs the oracle ----
    cpu = None
    cpu_context = None
    parity = None
    if not a.no_cpu:
        import oracle
        kc = ks[0]
        sample = np.arange(0, g.n, a.cpu_stride, dtype=np.int32)
        if order != dist.ORDER_DEGREE:
            Gd = dist.orient(rp, col, order=dist.ORDER_DEGREE)
        else:
            Gd = G
        per = torch.zeros(3 * g.n, dtype=torch.int64, device="cuda")
        dist.count(Gd, kc, cfg=dist.config(), per_root=per, stream=stream)
        torch.cuda.synchronize()
        per_h = per.cpu().numpy().view(np.uint64)
        threads = min(16, os.cpu_count() or 1)
        log("oracle sample: %d roots, %d threads" % (len(sample), threads))
        tc = time.perf_counter()
        want = oracle.count_roots(g.row_ptr, g.col, kc, sample, nthreads=threads)
        cpu_s = time.perf_counter() - tc
        got = [(int(per_h[3 * v]) | (int(per_h[3 * v + 1]) << 64), int(per_h[3 * v + 2])) for v in sample]
        parity = bool(got == want)
        sample_cliques = sum(c for c, _ in want)
        cpu = {"value": sample_cliques / cpu_s, "unit": "k-cliques/s", "cores": threads, "kind": "oracle",
               "sample": "k=%d, every %d-th vertex id as root (%d roots, %d cliques, %.1f s)" % (
                   kc, a.cpu_stride, len(sample), sample_cliques, cpu_s)}
        # context: the host CPU, the oracle on one thread and the pivot-based
        # reference, on a 16x smaller sample of the same roots
        small = sample[::16]
        t1 = time.perf_counter()
        w1 = oracle.count_roots(g.row_ptr, g.col, kc, small, nthreads=1)
        s1 = time.perf_counter() - t1
        t1 = time.perf_counter()
        wp = oracle.pivot_count_roots(g.row_ptr, g.col, kc, small, nthreads=threads)
        sp = time.perf_counter() - t1
        assert wp == w1 == [want[i] for i in range(0, len(sample), 16)], "oracle and pivot reference disagree"
        c1 = sum(c for c, _ in w1)
        cpu_context = {"cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
                       "sample": "k=%d, every %d-th vertex id as root (%d roots, %d cliques)" % (
                           kc, a.cpu_stride * 16, len(small), c1),
                       "oracle_1thread": {"value": c1 / s1, "unit": "k-cliques/s", "s": round(s1, 3)},
                       "pivot_%dthreads" % threads: {"value": c1 / sp, "unit": "k-cliques/s", "s": round(sp, 3)}}
        log("oracle on 1 thread: %.3g k-cliques/s; pivot reference on %d threads: %.3g k-cliques/s" % (
            c1 / s1, threads, c1 / sp))

    pivot = None
    if not a.no_pivot:
        pivot = run_pivot(a, dist, torch, G, g, results, log)
    listing = None
    if not a.no_listing:
        listing = run_listing(a, dist, torch, log)
    cfg3 = None
    if not a.no_cfg3:
        cfg3 = run_cfg3(a, dist, torch, log)
    batched = None
    if batch_graphs is not None:
        batched = run_batched(a, dist, torch, batch_specs, batch_graphs, log)
    serving = None
    if serve_inputs is not None:
        serving = run_serving(a, dist, torch, serve_inputs, log)

    line = {
        "metric": "k-cliques/sec at k=5..9 (plain vs batched); p50/p99 query latency in serving",
        "value": value,
        "unit": "k-cliques/s",
        "rate_kind": "counting rate: k-cliques counted (with their fingerprint), not enumerated, per second",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "plain per-graph: Chung-Lu n=%d, exponent 2.2, mean degree 20, cap 5000, "
                               "+200 planted K30, seed 2; orient (%s order) + count k=%s" % (
                                   g.n, a.order, ",".join(map(str, ks))),
                   "n": g.n, "m": g.m, "ks": ks},
        "per_k": [{"k": k, "count": results[k][0], "fp": results[k][1], "fingerprint": k in fp_ks,
                   "ms": float(np.median(per_k[k]["ms"])),
                   "kernel_ms": float(np.median(per_k[k]["kernel_ms"])),
                   "cliques_per_s": results[k][0] / (np.median(per_k[k]["ms"]) / 1e3),
                   "memo": {x: per_k[k]["stats"]["memo_" + x] for x in ("lookups", "hits", "inserts")},
                   "frames": per_k[k]["stats"]["frames"], "leaf_bits": per_k[k]["stats"]["leaf_bits"]}
                  for k in ks],
        "orient_ms": float(np.median(orient_ms)),
        "k_dnf": dnf,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_context": cpu_context,
        "parity_sampled_roots": parity,
        "pivot_all_k": pivot,
        "listing": listing,
        "dense_core_rmat": cfg3,
        "batched": batched,
        "serving": serving,
        "gen_s": gen_s,
    }
    s = json.dumps(line)
    print(s, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(s + "\n")


def run_pivot(a, dist, torch, G, g, results, log):
    """Pivot-based counting of every clique size in one pass (dist_count_all,
    k <= 9) on the same oriented graph: not part of the timed step; its
    totals must equal the search's at every k the step measured."""
    kmax = max(9, max(results))
    torch.cuda.synchronize()
    t = time.perf_counter()
    res, rc = dist.count_all(G, kmax)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    st = G.stats()
    same = all(res[k] == results[k] for k in results)
    log("pivot all-k (k <= %d): %.0f ms, tree nodes %d, same as the search: %s" % (kmax, dt * 1e3, st.frames, same))
    return {"workload": "Chung-Lu n=%d (the step's graph), every k <= %d in one pass" % (g.n, kmax),
            "ms": dt * 1e3, "kernel_ms": st.kernel_ms, "tree_nodes": st.frames, "leaves": st.leaf_bits,
            "counts": {str(k): [str(res[k][0]), str(res[k][1])] for k in range(kmax + 1)},
            "same_as_search": same, "status": rc}


def run_listing(a, dist, torch, log):
    """Listing (dist_list_ex, rows left in device memory and handed to a
    counting sink) on the small Chung-Lu graph (n = 10^4, 20 planted
    12-cliques): k = 4 (criterion (1) never holds: plain Listing) and k = 6
    with the Induced Subgraph Trie under criterion (1) and forced on every
    branch, against plain Listing.  Output-write roofline: 4k bytes per
    clique against the 8 TB/s of HBM."""
    import numpy as np
    from paper_2502_00317_amd import graphgen as gg
    g = gg.small_powerlaw()
    G = dist.orient(g.row_ptr, g.col)
    out = {"workload": "listing: Chung-Lu n=10,000, exponent 2.5, mean degree 8, cap 200, +20 planted K12, seed 1",
           "legs": []}
    for k, memo in ((4, 1), (6, 0), (6, 1), (6, 2)):
        times = []
        for _ in range(max(1, min(a.steps, 5))):
            seen = [0]

            def sink(ptr, n, kk):
                seen[0] += n
                return 0

            torch.cuda.synchronize()
            t = time.perf_counter()
            _, cnt, fp, rc = dist.list_cliques(G, k, cfg=dist.config(memo=memo), device_rows=True, raw_sink=sink)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
            assert seen[0] == cnt and rc == dist.OK
        st = G.stats()
        sec = float(np.median(times))
        gbs = cnt * 4 * k / sec / 1e9
        leg = {"k": k, "memo": memo, "cliques": cnt, "fp": fp, "ms": sec * 1e3, "cliques_per_s": cnt / sec,
               "bytes_written": cnt * 4 * k, "write_GBps": gbs, "write_frac_of_8TBps": gbs / 8000.0,
               "dense_frames": st.memo_lookups, "trie_nodes": st.memo_inserts, "retrievals": st.memo_hits,
               "retrieved_cliques": st.leaf_bits, "frames": st.frames}
        out["legs"].append(leg)
        log("listing k=%d memo=%d: %d cliques in %.2f ms (%.3g/s, %.2f GB/s written), %d retrieved" % (
            k, memo, cnt, sec * 1e3, cnt / sec, gbs, st.leaf_bits))
    G.free()
    return out


def run_cfg3(a, dist, torch, log):
    """The dense-core stress graph (R-MAT scale 22, edge factor 16, 10 planted
    60-cliques): orientation, then k = 6 and 8 by the search and every k <= 12
    by pivoting, each under a short deadline, and k = 6 again in degree order
    under a long one (the heavy roots' arcs as EdgeParallel units); a count
    that does not finish is reported as DNF."""
    from paper_2502_00317_amd import graphgen as gg
    t = time.time()
    g = gg.dense_core_rmat()
    gen_s = time.time() - t
    torch.cuda.synchronize()
    t = time.perf_counter()
    G = dist.orient(g.row_ptr, g.col, order=dist.ORDER_DEGENERACY)
    torch.cuda.synchronize()
    orient_ms = (time.perf_counter() - t) * 1e3
    info = G.info()
    out = {"workload": "R-MAT scale 22, ef 16, (0.57,0.19,0.19,0.05), +10 planted K60, seed 3",
           "n": g.n, "m": g.m, "gen_s": gen_s, "orient_ms": orient_ms, "degeneracy": info.order_bound,
           "max_outdeg": info.max_outdeg, "deadline_ms": a.cfg3_deadline_ms, "search": {}, "pivot": None}
    for k in (6, 8):
        try:
            c, f, rc = dist.count(G, k, cfg=dist.config(deadline_ms=a.cfg3_deadline_ms))
            out["search"][str(k)] = {"status": "finished", "count": str(c), "fp": str(f)}
        except dist.DistError as e:
            st = G.stats()
            out["search"][str(k)] = {"status": "DNF" if e.status == dist.E_CANCELLED else "error %d" % e.status,
                                     "roots_done": st.roots}
        log("dense-core R-MAT search k=%d: %s" % (k, out["search"][str(k)]["status"]))
    res, rc = dist.count_all(G, 12, cfg=dist.config(deadline_ms=a.cfg3_deadline_ms))
    st = G.stats()
    out["pivot"] = {"kmax": 12, "status": {dist.OK: "finished", dist.E_OVERFLOW: "finished (k=12 >= 2^64)",
                                           dist.E_CANCELLED: "DNF"}.get(rc, "error %d" % rc),
                    "roots_done": st.roots, "tree_nodes": st.frames}
    if rc in (dist.OK, dist.E_OVERFLOW):
        out["pivot"]["counts"] = {str(k): [str(res[k][0]), str(res[k][1])] for k in range(13)}
    log("dense-core R-MAT pivot k<=12: %s" % out["pivot"]["status"])
    G.free()
    if a.cfg3_k6_deadline_ms > 0:
        H = dist.orient(g.row_ptr, g.col, order=dist.ORDER_DEGREE)
        torch.cuda.synchronize()
        t = time.perf_counter()
        try:
            c, f, rc = dist.count(H, 6, cfg=dist.config(deadline_ms=a.cfg3_k6_deadline_ms))
            torch.cuda.synchronize()
            s = time.perf_counter() - t
            st = H.stats()
            out["k6_degree_order"] = {"status": "finished", "count": str(c), "fp": str(f), "s": s,
                                      "cliques_per_s": c / s, "kernel_ms": st.kernel_ms, "units": st.roots,
                                      "deadline_ms": a.cfg3_k6_deadline_ms}
        except dist.DistError as e:
            out["k6_degree_order"] = {"status": "DNF" if e.status == dist.E_CANCELLED else "error %d" % e.status,
                                      "deadline_ms": a.cfg3_k6_deadline_ms}
        log("dense-core R-MAT k=6 (degree order): %s" % out["k6_degree_order"]["status"])
        H.free()
    return out


def run_batched(a, dist, torch, specs, graphs, log):
    """4,096 Chung-Lu graphs (n ~ U{50..5000}, exponent ~ U[2.1, 3.0], mean
    degree ~ U[4, 40], 0-3 planted cliques of 8..25 vertices), each with its
    own k ~ U{3..12}: the plain path (one dist_count per pair) against the
    batched path (dist_count_batch: one persistent launch per width class,
    replayed from a captured HIP graph), both with fingerprints."""
    import numpy as np
    from paper_2502_00317_amd import autotune

    ks = [s["k"] for s in specs]
    t = time.perf_counter()
    G = [dist.orient(g.row_ptr, g.col) for g in graphs]
    torch.cuda.synchronize()
    orient_s = time.perf_counter() - t
    log("batched: oriented %d graphs in %.2f s" % (len(G), orient_s))
    cfg = dist.config()
    # plain: one call per pair
    t = time.perf_counter()
    plain = [dist.count(Gi, k, cfg=cfg)[:2] for Gi, k in zip(G, ks)]
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t
    total = sum(c for c, _ in plain)
    log("batched: plain loop %.2f s, %d cliques" % (plain_s, total))
    m_total = sum(g.m for g in graphs)
    db = autotune.TuningDB(os.path.join(a.state_dir, "autotune_db.json") if a.state_dir else None)
    best, report = autotune.tune_batch(dist, G, ks, m_total, db=db, log=log)
    bcfg = dist.config(**best)
    res, rc, _ = dist.count_batch(G, ks, cfg=bcfg, use_graph=True)
    times = []
    for _ in range(a.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r2, rc, dev_ms = dist.count_batch(G, ks, cfg=bcfg, use_graph=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        assert r2 == res
    batch_s = float(np.median(times))
    same = res == plain
    log("batched: %.3f s per batch (best %s), same as plain: %s" % (batch_s, best, same))
    # per-bucket switches: (width class, k band) buckets tuned alone, then the
    # whole batch in one captured run with each pair given its bucket's winner
    per_pair, buckets = autotune.tune_buckets(dist, G, ks, db=db, log=log, retune=True)
    res_t, rc, _ = dist.count_batch_tuned(G, ks, per_pair, use_graph=True)
    ttimes = []
    for _ in range(a.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r2, rc, dev_ms = dist.count_batch_tuned(G, ks, per_pair, use_graph=True)
        torch.cuda.synchronize()
        ttimes.append(time.perf_counter() - t)
        assert r2 == res_t
    tuned_s = float(np.median(ttimes))
    same_t = res_t == plain
    log("batched, per-bucket switches: %.3f s per batch (%.2fx the single best), same as plain: %s" % (
        tuned_s, batch_s / tuned_s, same_t))
    # the Induced Subgraph Trie shared by the consecutive roots of a wave
    # (soft bound tau, hard bound 2 tau), memo on, against the single best
    # switches (which may have the memo off)
    tau = 65536
    scfg = dist.config(trie_tau=tau, **dict(best, memo=1))
    res_s, rc, _ = dist.count_batch(G, ks, cfg=scfg, use_graph=True)
    stimes = []
    for _ in range(a.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r2, rc, _ = dist.count_batch(G, ks, cfg=scfg, use_graph=True)
        torch.cuda.synchronize()
        stimes.append(time.perf_counter() - t)
        assert r2 == res_s
    shared_s = float(np.median(stimes))
    log("batched, shared trie (tau %d): %.3f s per batch, same as plain: %s" % (tau, shared_s, res_s == plain))
    for Gi in G:
        Gi.free()
    best_s = min(batch_s, tuned_s)
    return {"workload": "batched: 4,096 Chung-Lu graphs n~U{50..5000}, exponent~U[2.1,3.0], "
                        "mean degree~U[4,40], 0-3 planted cliques of 8..25, k~U{3..12}, seed 4",
            "pairs": len(ks), "edges": m_total, "cliques": total,
            "value": total / best_s, "unit": "k-cliques/s", "ms_per_batch": best_s * 1e3,
            "plain_ms": plain_s * 1e3, "plain_value": total / plain_s,
            "speedup_vs_plain": plain_s / best_s, "orient_ms": orient_s * 1e3,
            "single_bucket": {"ms_per_batch": batch_s * 1e3, "switches": best, "candidates": report},
            "per_bucket": {"ms_per_batch": tuned_s * 1e3, "gain_vs_single_bucket": batch_s / tuned_s,
                           "buckets": {k: {"pairs": v["pairs"], "switches": v["switches"], "alone_ms": v["ms"]}
                                       for k, v in buckets.items()}},
            "shared_trie": {"trie_tau": tau, "memo": 1, "ms_per_batch": shared_s * 1e3,
                            "speedup_vs_single_best": batch_s / shared_s,
                            "same_as_plain": res_s == plain},
            "same_as_plain": same and same_t and res_s == plain, "fingerprint": True}


def run_serving(a, dist, torch, inputs, log):
    """Resident pool of 64 Chung-Lu graphs (n log-uniform in [1e4, 2e6],
    exponent U[2.2, 2.8], mean degree U[10, 30]) plus ad-hoc uploads (10% of
    queries, n log-uniform in [1e3, 5e4]); 2,000 (graph, k ~ U{3..12})
    queries arriving as a Poisson stream at 200 per second, each with a
    latency budget.  Served: continuous batching on two slots (an express
    lane with a short device budget and a bulk lane), memory-gated admission,
    per-query completion.  Plain: the same stream, one query at a time
    through the per-graph call with the whole device."""
    import numpy as np
    from paper_2502_00317_amd.serve import DeviceBackend, Query, Server, oriented_bytes, replay, summarize

    pool_specs, qspecs, pool_graphs, adhoc_graphs = inputs
    t = time.perf_counter()
    handles = {i: dist.orient(g.row_ptr, g.col) for i, g in enumerate(pool_graphs)}
    torch.cuda.synchronize()
    orient_s = time.perf_counter() - t
    pool_bytes = sum(oriented_bytes(g.n, g.m) for g in pool_graphs)
    mem_limit = pool_bytes + (1 << 30)
    log("serving: pool oriented in %.2f s, %.2f GB resident" % (orient_s, pool_bytes / 1e9))
    # warm-up before any clock starts, as a server does before it takes
    # traffic: every pool graph once at k = 3 (loads the kernels of every width
    # class the pool needs) and a few graphs of ad-hoc size oriented, counted
    # and freed (their blocks stay in the library's cache for later uploads)
    t = time.perf_counter()
    for h in handles.values():
        try:
            dist.count(h, 3, cfg=dist.config(deadline_ms=2000))
        except dist.DistError:
            pass
    for g in adhoc_graphs[:8]:
        W = dist.orient(g.row_ptr, g.col)
        try:
            dist.count(W, 4, cfg=dist.config(deadline_ms=2000))
        except dist.DistError:
            pass
        W.free()
    torch.cuda.synchronize()
    warm_s = time.perf_counter() - t
    log("serving: warm-up %.2f s" % warm_s)

    def queries():
        qs = []
        ai = 0
        for i, q in enumerate(qspecs):
            if "adhoc" in q:
                g = adhoc_graphs[ai]
                ai += 1
                qs.append(Query(qid=i, k=q["k"], t_arrival=q["t"], adhoc=(g.row_ptr, g.col),
                                deadline_ms=a.serve_deadline_ms))
            else:
                qs.append(Query(qid=i, k=q["k"], t_arrival=q["t"], graph=q["graph"],
                                deadline_ms=a.serve_deadline_ms))
        return qs

    out = {"workload": "serving: pool of 64 Chung-Lu graphs n log-U[1e4,2e6], exponent U[2.2,2.8], mean degree "
                       "U[10,30] + 10%% ad-hoc uploads n log-U[1e3,5e4]; 2,000 Poisson queries at 200/s, "
                       "k~U{3..12}, seed 5, latency budget %d ms per query" % a.serve_deadline_ms,
           "pool_edges": sum(g.m for g in pool_graphs), "pool_gb": pool_bytes / 1e9,
           "mem_limit_gb": mem_limit / 1e9, "orient_pool_s": orient_s,
           "warm_up": {"s": warm_s, "what": "each pool graph counted once at k = 3; 8 graphs of ad-hoc size "
                                            "oriented, counted at k = 4 and freed"}}
    nb = max(1, a.serve_bulk_slots)
    bulk_pct = max(1, (90 - a.serve_express_pct) // nb)  # 10% headroom: kernels of different widths co-reside
    modes = [("served", dict(slots=1 + nb, express_ms=a.serve_express_ms, express_batch_ms=a.serve_express_batch_ms,
                             shed_frac=a.serve_shed_frac), [a.serve_express_pct] + [bulk_pct] * nb,
              [{"budget_from_pair_start": 1}] + [{}] * nb),
             ("plain", dict(slots=1, plain=True), [100], [{}])]
    modes = [m for m in modes if m[0] in a.serve_modes.split(",")]
    ans = {}
    lat = {}
    # the served mode routes from a stored table, frozen, where one exists
    # (reproducible p50/p99); otherwise it learns online and its state is
    # written out for storing
    table = None
    if a.serve_router and os.path.exists(a.serve_router):
        with open(a.serve_router) as f:
            table = json.load(f)
    for name, kw, pcts, scfg in modes:
        be = DeviceBackend(slots=kw["slots"], grid_pcts=pcts, slot_cfgs=scfg)
        extra = dict(router_table=table, learn=table is None, pivot_k=a.serve_pivot_k) if name == "served" else {}
        srv = Server(be, handles, mem_limit=mem_limit, pool_bytes=pool_bytes, **kw, **extra)
        qs = queries()
        srv.start()
        replay(srv, qs, log=log)
        wall = srv.now()
        srv.stop()
        summ = summarize(qs, wall)
        sizes = [b[1] for b in srv.batches]
        summ.update({"slots": kw["slots"], "grid_pcts": pcts, "batches": len(srv.batches),
                     "mean_batch": float(np.mean(sizes)) if sizes else 0.0,
                     "max_batch": max(sizes) if sizes else 0, "peak_mem_gb": srv.peak_mem / 1e9,
                     "error_msgs": srv.errors[:3]})
        if name == "served":
            summ.update({"express_ms": srv.express_ms, "express_batch_ms": srv.express_batch_ms,
                         "moved_to_bulk": srv.demoted, "routed_to_bulk": srv.routed_bulk,
                         "heavy_keys": len(srv.heavy), "shed": srv.shed, "shed_frac": srv.shed_frac,
                         "router": ("stored table %s, frozen" % os.path.relpath(a.serve_router, ROOT))
                         if table is not None else "learned online",
                         "pivot_k": srv.pivot_k, "pivot_passes": srv.pivot_passes,
                         "pivot_slow_graphs": len(srv.pivot_slow)})
            if table is None and a.state_dir:
                with open(os.path.join(a.state_dir, "router_state.json"), "w") as f:
                    json.dump(srv.router_state(), f, indent=1, sort_keys=True)
        ans[name] = {(q.qid): (q.count, q.fp) for q in qs if q.status in ("ok", "overflow")}
        lat[name] = {q.qid: q.latency for q in qs if q.status in ("ok", "overflow")}
        if a.serve_trace:
            with open(a.serve_trace + "." + name + ".json", "w") as f:
                json.dump({"batches": srv.batches,
                           "queries": [[q.qid, q.graph, q.k, q.lane, q.moves, q.status, q.t_arrival, q.t_start,
                                        q.t_done, q.slot, q.batch_size] for q in qs]}, f)
        log("serving[%s]: p50 %.1f ms p99 %.1f ms (unfinished at their budget), %d/%d completed, %d DNF, "
            "%d shed, %.3g cliques/s" % (name, summ["p50_ms"], summ["p99_ms"], summ["completed"], summ["queries"],
                                         summ["dnf"], summ["shed"], summ["cliques_per_s"]))
        out[name] = summ
    if "served" in ans and "plain" in ans:
        both = set(ans["served"]) & set(ans["plain"])
        out["same_results_where_both_completed"] = all(ans["served"][i] == ans["plain"][i] for i in both)
        out["compared"] = len(both)
        if both:
            # latency percentiles of the two modes over the same queries
            out["both_completed"] = {m: {"p50_ms": float(np.percentile([lat[m][i] for i in both], 50) * 1e3),
                                         "p99_ms": float(np.percentile([lat[m][i] for i in both], 99) * 1e3)}
                                     for m in ("served", "plain")}
    for h in handles.values():
        h.free()
    return out


if __name__ == "__main__":
    main()
