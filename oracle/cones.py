"""Cone projection and absolute value (Definition 1) for K = R_+^{n_orth} x L_k1 x ... .

Test infrastructure only (see the package header).

The Lorentz cone L_k = {w : w_1 >= ||w_{2:k}||_2} (Sec. II, definition of K).
A size-one Lorentz cone is the half line R_+, so the orthant block is handled
as n_orth cones of size one.  The paper does not print the projection onto
L_k; the oracle uses the textbook closed form (e.g. Boyd & Vandenberghe,
Convex Optimization, exercise 8.3 / Parikh & Boyd, Proximal Algorithms 6.3.2):

    proj(v0, v) = (v0, v)                        if ||v|| <= v0
                = 0                              if ||v|| <= -v0
                = (v0 + ||v||)/2 * (1, v/||v||)  otherwise.
"""
from __future__ import annotations

from typing import Iterator, Sequence, Tuple

import numpy as np


def blocks(n_orth: int, soc_sizes: Sequence[int]) -> Iterator[Tuple[int, int]]:
    """Yield (start, size) of every Lorentz cone block of a vector in K.

    Orthant coordinates come first (each a cone of size one), then the
    second-order cones in list order."""
    for j in range(n_orth):
        yield j, 1
    off = n_orth
    for k in soc_sizes:
        yield off, int(k)
        off += int(k)


def proj_lorentz(v: np.ndarray) -> np.ndarray:
    """Euclidean projection of one block onto the Lorentz cone (Def. 1)."""
    v = np.asarray(v, dtype=np.float64)
    v0 = v[0]
    vb = v[1:]
    nv = float(np.linalg.norm(vb))
    if nv <= v0:
        return v.copy()
    if nv <= -v0:
        return np.zeros_like(v)
    a = 0.5 * (v0 + nv)
    out = np.empty_like(v)
    out[0] = a
    out[1:] = (a / nv) * vb
    return out


def proj_K(v: np.ndarray, n_orth: int, soc_sizes: Sequence[int]) -> np.ndarray:
    """proj_K(v) = argmin_{u in K} ||u - v||_2, blockwise (Def. 1)."""
    v = np.asarray(v, dtype=np.float64)
    out = np.empty_like(v)
    out[:n_orth] = np.maximum(v[:n_orth], 0.0)
    off = n_orth
    for k in soc_sizes:
        k = int(k)
        out[off:off + k] = proj_lorentz(v[off:off + k])
        off += k
    if off != v.shape[0]:
        raise ValueError("cone sizes do not add up to the vector length")
    return out


def abs_K(v: np.ndarray, n_orth: int, soc_sizes: Sequence[int]) -> np.ndarray:
    """abs_K(v) = 2 proj_K(v) - v (Def. 1)."""
    return 2.0 * proj_K(v, n_orth, soc_sizes) - np.asarray(v, dtype=np.float64)


def dist_K(v: np.ndarray, n_orth: int, soc_sizes: Sequence[int]) -> float:
    """Euclidean distance from v to K."""
    return float(np.linalg.norm(np.asarray(v, dtype=np.float64) - proj_K(v, n_orth, soc_sizes)))


def e_K(n_orth: int, soc_sizes: Sequence[int]) -> np.ndarray:
    """The cone's identity element: 1 on every orthant coordinate and
    (1, 0, ..., 0) on every Lorentz block."""
    n = n_orth + int(np.sum(soc_sizes)) if len(soc_sizes) else n_orth
    e = np.zeros(n)
    for start, _ in blocks(n_orth, soc_sizes):
        e[start] = 1.0
    return e
