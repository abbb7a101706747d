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

Those terms are normalised by the norms of b and c, so a point that meets
them can still carry a larger relative error in the objective.  For any
optimal pair (y*, z*) of the dual (Sec. II), with r_p = A x - b and
r_d = A^T y + z - c, expanding c = A^T y* + z* and b = A x - r_p gives the
identity

    c^T x - p* = z*^T x + y*^T r_p,

so |c^T x - p*| <= sum_j |x_j z*_j| over the orthant + |sum_C x_C^T z*_C|
over the Lorentz cones + |y*^T r_p| (for x in K each cone's term is >= 0,
so the cone sum equals the sum of its absolute values).  The estimate takes
that bound at the current (y, z):

    eps_obj = (sum_j |x_j z_j| + |sum_C x_C^T z_C| + |y^T r_p|) / (1 + |c^T x|)

Replacing (y*, z*) by (y, z) changes the orthant terms by products of two
small quantities, since x* and z* are complementary coordinate by
coordinate: |x_j| is small where z*_j is not, and |z_j| itself is the error
where x*_j is not.  The orthant's absolute values keep complementarity terms
of opposite signs (x or z slightly outside the cone) from cancelling.  Within
a Lorentz cone x*_C and z*_C are both nonzero on the boundary, and x_C^T z_C
carries first-order errors of either sign in every cone: summed in absolute
value over thousands of cones they stay far above the objective's error (a
served SOCP with 9000 cones at KKT 2e-7: 1.4e-4 against an error near 1e-6),
so the cone terms are summed with their signs.  The row sum stays signed
too: the residual r_p of a first-order method is spread over the rows, and
row-by-row absolute values would count it about sqrt(m) times over.  The
estimate still bounds the weak-duality form |c^T x - b^T y + r_d^T x| =
|x^T z + y^T r_p| and |y^T r_p|.  `objective_bounds` returns the exact
two-sided weak-duality bounds for a known optimum, used to pin the estimate.

`dual_multiplier_ls` gives the multiplier implicit in eq. stopcri's dual
objective (A^dagger b)^T (c - z) = b^T (A A^T)^+ A (c - z).
"""
from __future__ import annotations

from typing import Dict, Sequence

import numpy as np
import scipy.sparse as sp

from .cones import blocks, dist_K
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
    rp = A @ x - b
    rd = A.T @ y + z - c
    eps_p = float(np.linalg.norm(rp)) / (1.0 + float(np.linalg.norm(b)))
    eps_d = float(np.linalg.norm(rd)) / (1.0 + float(np.linalg.norm(c)))
    eps_g = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj))
    eps_k = max(dist_K(x, n_orth, soc_sizes), dist_K(z, n_orth, soc_sizes)) / (
        1.0 + max(float(np.linalg.norm(x)), float(np.linalg.norm(z))))
    xz_orth = float(np.sum(np.abs(x[:n_orth] * z[:n_orth])))
    xz_soc = sum(float(x[st:st + k] @ z[st:st + k]) for st, k in blocks(n_orth, soc_sizes) if st >= n_orth)
    eps_obj = (xz_orth + abs(xz_soc) + abs(float(rp @ y))) / (1.0 + abs(pobj))
    return {"eps_p": eps_p, "eps_d": eps_d, "eps_g": eps_g, "eps_k": eps_k,
            "kkt": max(eps_p, eps_d, eps_g, eps_k), "pobj": pobj, "dobj": dobj, "eps_obj": eps_obj}


def objective_bounds(A: sp.csr_matrix, b: np.ndarray, c: np.ndarray, x: np.ndarray, y: np.ndarray,
                     z: np.ndarray, x_opt: np.ndarray, y_opt: np.ndarray):
    """(lower, upper) with lower <= c^T x - p* <= upper for x, z in K and an
    optimal pair (x_opt, y_opt): lower = y*^T r_p, upper = c^T x - b^T y +
    r_d^T x* (weak duality, see the module header)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    rp = A @ x - np.asarray(b, dtype=np.float64)
    rd = A.T @ y + z - np.asarray(c, dtype=np.float64)
    gap = float(np.asarray(c) @ x) - float(np.asarray(b) @ y)
    return float(np.asarray(y_opt) @ rp), gap + float(rd @ np.asarray(x_opt))


def dual_multiplier_ls(A: sp.csr_matrix, c: np.ndarray, z: np.ndarray) -> np.ndarray:
    """y = (A A^T)^+ A (c - z): the least-squares multiplier of A^T y = c - z."""
    P = RangeProjector(A, np.ones(A.shape[1]))
    return P.solve_normal(P.B @ (np.asarray(c, dtype=np.float64) - np.asarray(z, dtype=np.float64)))
