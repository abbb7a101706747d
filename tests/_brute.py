"""Brute-force optimum of a tiny standard-form LP by enumerating every basis
(vertex enumeration).  Independent of the oracle's iteration."""
import itertools

import numpy as np


def lp_vertex_optimum(A, b, c, tol=1e-10):
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    best = None
    for basis in itertools.combinations(range(n), m):
        B = A[:, basis]
        if abs(np.linalg.det(B)) < 1e-12:
            continue
        xb = np.linalg.solve(B, b)
        if (xb >= -tol).all():
            x = np.zeros(n)
            x[list(basis)] = xb
            v = float(c @ x)
            if best is None or v < best[0]:
                best = (v, basis, x)
    return best
