"""KKT residuals of the primal/dual pair (Sec. II, eqs. prob_primal / prob_dual).

Test infrastructure only (see the package header).

The paper stops its runs by comparing against a competing solver (eq.
stopcri); without one, the oracle measures the optimality conditions the
appendix's proof establishes (A x = b; c - z in range(A^T) through y;
x^T z = 0; x, z in K) as relative errors:

    eps_p = ||A x - b|| / (1 + ||b||)
    eps_d = ||A^T y + z - c|| / (1 + ||c||)
    eps_g = |c^T x - b^T y| / (1 + |c^T x| + |b^T y|)
    eps_K = max(dist(x, K), dist(z, K)) / (1 + max(||x||, ||z||))
    kkt   = max(eps_p, eps_d, eps_g, eps_K)

`dual_multiplier_ls` gives the multiplier implicit in eq. stopcri's dual
objective (A^dagger b)^T (c - z) = b^T (A A^T)^+ A (c - z).
"""
from __future__ import annotations

from typing import Dict, Sequence

import numpy as np
import scipy.sparse as sp

from .cones import dist_K
from .subspace import RangeProjector


def kkt_errors(A: sp.csr_matrix, b: np.ndarray, c: np.ndarray, n_orth: int, soc_sizes: Sequence[int],
               x: np.ndarray, y: np.ndarray, z: np.ndarray) -> Dict[str, float]:
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    pobj = float(c @ x)
    dobj = float(b @ y)
    eps_p = float(np.linalg.norm(A @ x - b)) / (1.0 + float(np.linalg.norm(b)))
    eps_d = float(np.linalg.norm(A.T @ y + z - c)) / (1.0 + float(np.linalg.norm(c)))
    eps_g = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
    eps_k = max(dist_K(x, n_orth, soc_sizes), dist_K(z, n_orth, soc_sizes)) / (
        1.0 + max(float(np.linalg.norm(x)), float(np.linalg.norm(z))))
    return {"eps_p": eps_p, "eps_d": eps_d, "eps_g": eps_g, "eps_k": eps_k,
            "kkt": max(eps_p, eps_d, eps_g, eps_k), "pobj": pobj, "dobj": dobj}


def dual_multiplier_ls(A: sp.csr_matrix, c: np.ndarray, z: np.ndarray) -> np.ndarray:
    """y = (A A^T)^+ A (c - z): the least-squares multiplier of A^T y = c - z."""
    P = RangeProjector(A, np.ones(A.shape[1]))
    return P.solve_normal(P.B @ (np.asarray(c, dtype=np.float64) - np.asarray(z, dtype=np.float64)))
