"""The oracle still reproduces its committed c1 fixture bit for bit."""
import json
import os

import numpy as np

import oracle as O
from meshgen import config_case

GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_c1.json")


def test_oracle_reproduces_c1_fixture():
    gold = json.load(open(GOLD))
    c = config_case("c1")
    A = O.Ldu.from_case(c)
    p = O.pcg(A, c.rhs[0], tol=1e-8)
    assert p.iterations == gold["pcg"]["iterations"]
    assert np.array_equal(p.history, np.array(gold["pcg"]["history"]))
    g = O.Gamg(A)
    s = g.solve(c.rhs[0], tol=1e-8)
    assert s.iterations == gold["gamg"]["cycles"]
    assert np.array_equal(s.history, np.array(gold["gamg"]["history"]))
    assert [g.level(l).n for l in range(g.n_levels)] == gold["gamg"]["level_cells"]
