"""Worked integer example (tests/golden/worked_2x3x2_r2.txt).

Row M2 0 can be checked by hand: with c = 0, sum over (i0, i1) of
X(i0,i1,0) U_0(i0,0) U_1(i1,0) = (1+6) + (6+24) + (-5-18) = 14.
"""
import os

import numpy as np

import brute
from oracle import oracle as O

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load():
    rows = {}
    with open(os.path.join(HERE, "worked_2x3x2_r2.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tag, i, *vals = line.split()
            rows.setdefault(int(tag[1:]), {})[int(i)] = [float(v) for v in vals]
    return {n: np.array([r[i] for i in sorted(r)]) for n, r in rows.items()}


DIMS = (2, 3, 2)
X = np.arange(1, 13, dtype=np.float64)
U = [np.array([[1, 2], [3, -1]], dtype=np.float64),
     np.array([[1, 0], [2, 1], [-1, 3]], dtype=np.float64),
     np.array([[2, 1], [0, -2]], dtype=np.float64)]


def test_worked_example():
    g = load()
    assert g[2][0, 0] == 14.0
    for n in range(3):
        np.testing.assert_array_equal(O.mttkrp(X, DIMS, U, n), g[n])
        np.testing.assert_array_equal(brute.mttkrp(X, DIMS, U, n), g[n])
