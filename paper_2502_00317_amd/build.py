"""Compile libdist.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdist.so")
SOURCES = ["api.cpp", "memcache.cpp", "orient.hip", "search.hip", "ist.hip", "pivot.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = False) -> str:
    """Compiles every source to an object in parallel, then links libdist.so."""
    from concurrent.futures import ThreadPoolExecutor
    tmp = LIB + ".tmp%d" % os.getpid()
    common = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wall", "-Wno-unused-function",
              "-I", os.path.join(HERE, "..", "include")]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        res = subprocess.run(cmd, capture_output=True, text=True)
        out = "\n".join(l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l)
        return res.returncode, out

    objs = [os.path.join(objdir, f + ".%d.o" % os.getpid()) for f in SOURCES]
    cmds = [common + ["-c", "-o", o, os.path.join(CSRC, f)] for f, o in zip(SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        results = list(ex.map(run, cmds))
    for (rc, out), f in zip(results, SOURCES):
        if rc != 0:
            raise RuntimeError("hipcc failed on %s:\n%s" % (f, out))
        if verbose and out.strip():
            print(out, file=sys.stderr)
    rc, out = run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    for o in objs:
        os.remove(o)
    if rc != 0:
        raise RuntimeError("link failed:\n" + out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
