"""Writes rmat_s22_degeneracy.json: the degeneracy of the dense-core stress
graph (R-MAT scale 22, edge factor 16, (0.57, 0.19, 0.19, 0.05), 10 planted
60-cliques, seed 3) as computed by the CPU oracle (minimum-degree removal).
Run from the repository root: python tests/golden/make_rmat_degeneracy.py"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))


def main():
    import oracle
    from paper_2502_00317_amd import graphgen as gg
    g = gg.dense_core_rmat()
    d, _ = oracle.degeneracy(g.row_ptr, g.col)
    out = {"graph": "R-MAT scale 22, edge factor 16, (0.57,0.19,0.19,0.05), +10 planted K60, seed 3",
           "n": g.n, "m": g.m, "degeneracy": d, "source": "oracle.degeneracy (oracle/oracle.c)"}
    with open(os.path.join(HERE, "rmat_s22_degeneracy.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
