"""Stored values under tests/golden/:

  * gll_lobatto.json: the published closed forms of the Gauss-Lobatto nodes
    and weights (orders 2-6), evaluated here at 30 digits, against the
    oracle's GLL rule and against the library's host FE builder (nodes and
    nodal weights of one and two cells);
  * oracle_24cube.json (written by tests/golden/make_golden.py from the
    oracle only): the oracle still reproduces its own stored FP64 energies
    (a change to its arithmetic shows here).
No GPU."""
import json
import os

import mpmath
import numpy as np
import pytest

from oracle import txe_oracle as O
from paper_2401_04189_amd import txe, workloads as W

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def lobatto(p):
    g = json.load(open(os.path.join(GOLD, "gll_lobatto.json")))["orders"][str(p)]
    mpmath.mp.dps = 30
    # the fixture's closed forms use only numbers, + - * /, parentheses and sqrt;
    # they are evaluated in 30-digit arithmetic with nothing else in scope
    env = {"__builtins__": {}, "sqrt": mpmath.sqrt, "one": mpmath.mpf(1)}
    ev = lambda e: mpmath.mpf(eval(e.replace("/", "*one/"), env))  # noqa: E731,S307
    return np.array([float(ev(e)) for e in g["nodes"]]), np.array([float(ev(e)) for e in g["weights"]])


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6])
def test_published_lobatto_rule(p):
    s, w = lobatto(p)
    assert abs(w.sum() - 2.0) <= 1e-15
    so, wo = O.gll_points(p)
    assert np.abs(so - s).max() <= 1e-15 and np.abs(wo - w).max() <= 1e-15
    # the library: one cell [-1, 1] holds the interior nodes with their weights
    x, q = txe.fe_mesh_1d([-1.0, 1.0], p)
    assert np.abs(x - s[1:-1]).max() <= 1e-15 and np.abs(q - w[1:-1]).max() <= 1e-15
    # two cells [-1, 1], [1, 3]: the shared node carries both end weights
    x2, q2 = txe.fe_mesh_1d([-1.0, 1.0, 3.0], p)
    assert abs(x2[p - 1] - 1.0) <= 1e-15 and abs(q2[p - 1] - 2 * w[0]) <= 1e-15


def test_oracle_reproduces_its_stored_energies():
    gold = json.load(open(os.path.join(GOLD, "oracle_24cube.json")))
    s = W.build_config("cfg1")
    st = O.Setup.from_system(s)
    pairs = {}
    vx, ex = O.apply(s.psi.numpy(), st, pairs_out=pairs)
    N = s.N
    ep = np.array([pairs[(i, j)] for i in range(N) for j in range(i, N)])
    assert abs(ex - gold["E_x"]) <= 1e-13 * abs(gold["E_x"])
    assert np.abs(ep - np.array(gold["e_pairs_upper_row_major"])).max() <= 1e-13 * np.abs(ep).max()
