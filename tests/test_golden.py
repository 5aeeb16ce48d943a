"""The oracle against small worked examples derived by hand (tests/golden/)."""
import math
import os

import numpy as np

from oracle import prior
from oracle.layout import AxisLayout

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if line:
                rows.setdefault(line[0], []).append([float(v) for v in line[1:]])
    return rows


def test_axis_layout_worked_example():
    g = _read("axis_layout_M40_T2_p20_o4_r2_G2.txt")
    A = AxisLayout(M=40, T=2, p=20, o=4, r=2, G=2)
    for a, s, e in g["block"]:
        assert A.block(int(a)) == (int(s), int(e))
    for a, s, e in g["support"]:
        assert A.support(int(a)) == (int(s), int(e))
    for row in g["omega"]:
        a, w = int(row[0]), np.array(row[1:])
        assert np.array_equal(A.omega(a), w)          # dyadic values: exact
    coords = np.array(g["coords"][0])
    for row in g["tent"]:
        k, w = int(row[0]), np.array(row[1:])
        assert np.allclose(A.tent(k, coords), w, rtol=0, atol=1e-15)


def test_smoothed_tv_worked_example():
    g = _read("smoothed_tv_2x2.txt")
    x = np.array(g["x"][0]).reshape(2, 2)
    eps = g["eps"][0][0]
    for bc in ("neumann", "circular"):
        pairs = np.array(g[bc + "_pairs"][0]).reshape(4, 2)
        by_hand = sum(math.sqrt(gh * gh + gv * gv + eps * eps) - eps for gh, gv in pairs)
        assert abs(by_hand - g[bc][0][0]) <= 1e-14
        assert abs(prior.value(x, "tv", eps, bc) - by_hand) <= 1e-13
