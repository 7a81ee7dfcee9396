"""Write tests/golden/oracle_c1.json from the CPU oracle only.

The stored values are the oracle's results on the 32^3 manufactured-solution
workload (diagonal PCG and GAMG, FP64, tol 1e-8); tests use them as a
regression fixture and the GPU tests compare iteration counts against them.
Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from meshgen import config_case  # noqa: E402


def main():
    c = config_case("c1")
    A = O.Ldu.from_case(c)
    p = O.pcg(A, c.rhs[0], tol=1e-8)
    g = O.Gamg(A)
    s = g.solve(c.rhs[0], tol=1e-8)
    out = {
        "workload": "32^3 FD Laplacian, Dirichlet x=0 (half cell), b = A p_h",
        "pcg": {"tol": 1e-8, "iterations": p.iterations,
                "history": [float(v) for v in p.history],
                "true_residual": p.true_residual},
        "gamg": {"tol": 1e-8, "cycles": s.iterations,
                 "history": [float(v) for v in s.history],
                 "level_cells": [g.level(l).n for l in range(g.n_levels)],
                 "level_faces": [g.level(l).nf for l in range(g.n_levels)]},
    }
    with open(os.path.join(HERE, "oracle_c1.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
