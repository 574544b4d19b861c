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
