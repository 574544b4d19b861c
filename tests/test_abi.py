"""The C-ABI library loads and exports every symbol include/dist.h declares
(CPU only: no compute calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dist.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(dist_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("dist_orient", "dist_count", "dist_list", "dist_count_batch",
                 "dist_graph_free", "dist_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2502_00317_amd import dist
    lib = ctypes.CDLL(dist.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror_and_config_defaults():
    from paper_2502_00317_amd import dist
    assert dist.strerror(dist.OK) == "ok"
    assert "k" in dist.strerror(dist.E_K)
    c = dist.config()
    assert (c.memo, c.prune, c.fingerprint, c.deadline_ms) == (1, 1, 1, 0)


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C layout: every
    field's offset and each struct's size, as gcc lays them out."""
    import subprocess
    from paper_2502_00317_amd import dist
    mirrors = {"dist_config": dist.Config, "dist_result": dist.Result, "dist_stats": dist.Stats,
               "dist_pair_switches": dist.PairSwitches, "dist_graph_info": dist.GraphInfo}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "dist.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (cname, cname))
        for f in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f[0], cname, f[0]))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict()
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    for cname, py in mirrors.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])
