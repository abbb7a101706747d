"""Textbook Douglas-Rachford splitting (Sec. III-A.1), used only as a pin.

Test infrastructure only (see the package header).

Problem eq. prob_primal is split as f + g with f the indicator of K and
g(x) = mu c^T x on {A x = b} (+inf elsewhere).  DR iterates

    x <- prox_f(zeta) = proj_K(zeta)
    zeta <- zeta + prox_g(2 x - zeta) - x

prox_g(v) = argmin_{A x = b} mu c^T x + ||x - v||^2 / 2 is computed here
from its own optimality system [I A^T; A 0] [x; lam] = [v - mu c; b]
(dense least squares), independently of the oracle's subspace projector.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from .cones import proj_K


def prox_affine_linear(A: np.ndarray, b: np.ndarray, c: np.ndarray, mu: float, v: np.ndarray) -> np.ndarray:
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    K = np.zeros((n + m, n + m))
    K[:n, :n] = np.eye(n)
    K[:n, n:] = A.T
    K[n:, :n] = A
    rhs = np.concatenate([np.asarray(v) - mu * np.asarray(c), np.asarray(b)])
    sol = np.linalg.lstsq(K, rhs, rcond=None)[0]
    return sol[:n]


def douglas_rachford(A: np.ndarray, b: np.ndarray, c: np.ndarray, n_orth: int, soc_sizes: Sequence[int],
                     mu: float, zeta0: np.ndarray, iters: int) -> List[np.ndarray]:
    """Return the DR variables zeta^1..zeta^iters."""
    zeta = np.asarray(zeta0, dtype=np.float64).copy()
    out = []
    for _ in range(iters):
        x = proj_K(zeta, n_orth, soc_sizes)
        zeta = zeta + prox_affine_linear(A, b, c, mu, 2.0 * x - zeta) - x
        out.append(zeta.copy())
    return out
