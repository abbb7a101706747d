"""Diagonal preconditioning of the data (Sec. III) and Algorithm 2 on the
preconditioned problem, in FP64.

Test infrastructure only (see the package header).

Sec. III rescales the data as  A_hat = D A E,  b_hat = D b,  c_hat = E c  with
the proxy variables  x_hat = E^{-1} x  and  z_hat = E z  (D, E positive
diagonal), and compares adaptive conditioning against the D, E that a
Sinkhorn-Knopp equilibration for l2 norms gives (the worked example of
Sec. III).  The paper cites a regularized variant of that method without its
regularization, and its printed factors for the example (E a multiple of the
identity) cannot be reproduced from the text: they are not used here.

The reading taken (the same one the GPU solver follows) is the plain l2
Sinkhorn-Knopp balancing of the squared entries.  With u = D^2 and v = E^2,
starting from v = 1, each sweep sets, rows first,

    u_i = 1 / sum_j a_ij^2 v_j             (every row of D A E: unit l2 norm)
    v_j = (m/n) / sum_i a_ij^2 u_i          (every column: l2 norm sqrt(m/n))

so that at the fixed point both conditions hold at once (the column target
m/n makes the two agree on the Frobenius norm, sum of squares = m).  On a
second-order cone E must be a constant (the Lorentz cone is invariant only
under a scaling that is the same on all of its coordinates), so a cone of k
coordinates takes v = (m/n) k / sum_{j in cone} sum_i a_ij^2 u_i: its columns
get mean square norm m/n.  A row or a column (or a whole cone) with no
nonzero keeps u = 1 / v = 1.

Algorithm 2 then runs unchanged on the preconditioned problem (its own O on
top, in the scaled space); the solution maps back as x = E x_hat,
z = E^{-1} z_hat, y = D y_hat.  In the original variables that run is
Algorithm 2 with the column scaling E O_hat: the iterate s is the same, and a
conditioning event takes the ratio of steps 5-10 from x_hat, z_hat, i.e. o / E^2.
"""
from __future__ import annotations

from typing import Dict, Sequence, Tuple

import numpy as np
import scipy.sparse as sp

from .alg2 import LP_SCHEDULE, LP_T, Algorithm2, Schedule
from .cones import blocks


def sinkhorn_knopp_l2(A, n_orth: int, soc_sizes: Sequence[int], sweeps: int) -> Tuple[np.ndarray, np.ndarray]:
    """(d, e): the diagonals of D and E after `sweeps` Sinkhorn-Knopp sweeps
    on the squared entries of A (module header)."""
    A = sp.csr_matrix(A, dtype=np.float64)
    m, n = A.shape
    S = A.multiply(A).tocsr()  # a_ij^2
    ST = S.T.tocsr()
    v = np.ones(n)
    u = np.ones(m)
    target = m / n
    cones = list(blocks(n_orth, soc_sizes))
    for _ in range(int(sweeps)):
        rs = S @ v
        u = np.where(rs > 0, 1.0 / np.where(rs > 0, rs, 1.0), 1.0)
        cs = ST @ u
        for start, k in cones:
            tot = float(cs[start:start + k].sum())
            v[start:start + k] = target * k / tot if tot > 0 else 1.0
    return np.sqrt(u), np.sqrt(v)


class EquilibratedAlgorithm2:
    """Algorithm 2 run literally on (D A E, D b, E c) (Sec. III scaling), with
    the solution mapped back to the original variables."""

    def __init__(self, A, b, c, n_orth: int, soc_sizes: Sequence[int], d: np.ndarray, e: np.ndarray,
                 mu: float = 1.0, t: float = LP_T, schedule: Schedule = LP_SCHEDULE, method: str = "auto"):
        self.A = sp.csr_matrix(A, dtype=np.float64)
        self.b = np.asarray(b, dtype=np.float64)
        self.c = np.asarray(c, dtype=np.float64)
        self.d = np.asarray(d, dtype=np.float64)
        self.e = np.asarray(e, dtype=np.float64)
        A_hat = sp.diags(self.d) @ self.A @ sp.diags(self.e)
        self.inner = Algorithm2(A_hat, self.d * self.b, self.e * self.c, n_orth, soc_sizes, mu=mu, t=t,
                                schedule=schedule, method=method)

    def step(self) -> None:
        self.inner.step()

    @property
    def l(self) -> int:
        return self.inner.l

    @property
    def s(self) -> np.ndarray:
        return self.inner.s

    @property
    def x(self) -> np.ndarray:
        return self.e * self.inner.x

    @property
    def z(self) -> np.ndarray:
        return self.inner.z / self.e

    @property
    def O(self) -> np.ndarray:
        """The column scaling of the original A that the scaled run amounts to."""
        return self.e * self.inner.O

    def dual_multiplier(self) -> np.ndarray:
        return self.d * self.inner.dual_multiplier()

    def kkt(self) -> Dict[str, float]:
        from .kkt import kkt_errors

        return kkt_errors(self.A, self.b, self.c, self.inner.n_orth, self.inner.soc_sizes, self.x,
                          self.dual_multiplier(), self.z)
