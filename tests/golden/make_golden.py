"""Writes the small worked-example fixture used by test_golden.py.

The expected values come only from the FP64 oracle in oracle/.  The inputs
are small integers, so every product and sum is exact in double precision
and the fixture can also be checked by hand against the definition of
MTTKRP in Section 2.2 of the paper.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from oracle import oracle as O  # noqa: E402

DIMS = (2, 3, 2)
R = 2
X = np.arange(1, 13, dtype=np.float64)              # storage order, mode 0 fastest
U = [np.array([[1, 2], [3, -1]], dtype=np.float64),
     np.array([[1, 0], [2, 1], [-1, 3]], dtype=np.float64),
     np.array([[2, 1], [0, -2]], dtype=np.float64)]


def main():
    path = os.path.join(HERE, "worked_2x3x2_r2.txt")
    with open(path, "w") as f:
        f.write("# dims (mode 0 fastest): %s\n" % " ".join(map(str, DIMS)))
        f.write("# X in storage order: %s\n" % " ".join("%g" % v for v in X))
        for k, u in enumerate(U):
            f.write("# U_%d rows: %s\n" % (k, " | ".join(" ".join("%g" % v for v in row) for row in u)))
        for n in range(len(DIMS)):
            M = O.mttkrp(X, DIMS, U, n)
            for i in range(DIMS[n]):
                f.write("M%d %d %s\n" % (n, i, " ".join("%.17g" % v for v in M[i])))
    print("wrote", path)


if __name__ == "__main__":
    main()
