"""Projection onto the subspace range((A O)^T) and the pseudo-inverse (A O)^dagger.

Test infrastructure only (see the package header).

Algorithms 1 and 2 use the subspace  A_hat = range{(A O)^T}  (Alg. 1 step 1,
Alg. 2 step 12), the reflection  abs_{A_hat}(v) = 2 proj_{A_hat}(v) - v
(Def. 1 applied to a subspace) and the vector (A O)^dagger b (Alg. 2 step 13).

Reading of the dagger (the notation list calls it a pseudo-inverse of the
transpose, while the algorithms apply it to b in R^m and write A^dagger A
for the projector onto range(A^T)): A^dagger = pinv(A) = A^T (A A^T)^+, an
n x m matrix.  With B = A O:

    proj_{range B^T}(v) = B^T (B B^T)^+ B v,      B^dagger b = B^T (B B^T)^+ b.

Two ways of applying (B B^T)^+, both plain library routines:
  * "exact": dense Cholesky of B B^T after dropping the all-zero rows (which
    contribute nothing to the range; consistency requires b_i = 0 there);
    a symmetric-eigendecomposition pseudo-inverse if Cholesky fails.
  * "pcg": SciPy's conjugate-gradient solver on B B^T with its diagonal as
    preconditioner, to a relative residual of 1e-12 (for problems too large
    for a dense factorisation).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

EXACT_MAX_ROWS = 4000


class RangeProjector:
    """Orthogonal projector onto range(B^T) with B = A diag(O)."""

    def __init__(self, A: sp.csr_matrix, O: np.ndarray, method: str = "auto", rtol: float = 1e-12):
        A = sp.csr_matrix(A, dtype=np.float64)
        O = np.asarray(O, dtype=np.float64)
        self.B = sp.csr_matrix(A @ sp.diags(O))  # post-multiplication by O (Alg. 2 step 12)
        self.m, self.n = self.B.shape
        if method == "auto":
            method = "exact" if self.m <= EXACT_MAX_ROWS else "pcg"
        self.method = method
        self.rtol = rtol
        row_nnz = np.diff(self.B.indptr)
        sq = np.asarray(self.B.multiply(self.B).sum(axis=1)).ravel()
        self.live = np.nonzero((row_nnz > 0) & (sq > 0))[0]
        if method == "exact":
            Bl = self.B[self.live]
            G = (Bl @ Bl.T).toarray()
            try:
                self._chol = sla.cho_factor(G, lower=True, check_finite=True)
                self._pinv = None
            except np.linalg.LinAlgError:
                self._chol = None
                w, V = np.linalg.eigh(G)
                cut = w.max() * G.shape[0] * np.finfo(np.float64).eps
                winv = np.where(w > cut, 1.0 / np.where(w > cut, w, 1.0), 0.0)
                self._pinv = (V * winv) @ V.T
        elif method == "pcg":
            diag = sq.copy()
            diag[diag == 0] = 1.0  # an empty row keeps a unit diagonal
            self._jac = 1.0 / diag
            self._warm = None
        else:
            raise ValueError(f"unknown method {method}")
        self.cg_iters = 0

    def solve_normal(self, rhs: np.ndarray, x0: np.ndarray | None = None) -> np.ndarray:
        """A solution w of (B B^T) w = rhs (rhs must lie in range(B))."""
        rhs = np.asarray(rhs, dtype=np.float64)
        if self.method == "exact":
            out = np.zeros(self.m)
            r = rhs[self.live]
            if self._chol is not None:
                out[self.live] = sla.cho_solve(self._chol, r)
            else:
                out[self.live] = self._pinv @ r
            return out
        B = self.B
        op = spla.LinearOperator((self.m, self.m), matvec=lambda v: B @ (B.T @ v), dtype=np.float64)
        M = spla.LinearOperator((self.m, self.m), matvec=lambda v: self._jac * v, dtype=np.float64)
        count = [0]

        def cb(_):
            count[0] += 1

        w, info = spla.cg(op, rhs, x0=x0, rtol=self.rtol, atol=0.0, maxiter=20 * self.m, M=M, callback=cb)
        self.cg_iters += count[0]
        if info != 0:
            raise RuntimeError(f"oracle PCG did not reach rtol={self.rtol} (info={info})")
        return w

    def normal_pinv(self) -> np.ndarray:
        """The m x m matrix (B B^T)^+ written out: on the rows of B that are not
        all zero the inverse of their Gram matrix, zero on the empty rows (they
        add nothing to range(B^T)).  Dense; for the exact method only."""
        if self.method != "exact":
            raise ValueError("normal_pinv needs the exact method")
        X = np.zeros((self.m, self.m))
        k = len(self.live)
        if self._chol is not None:
            inner = sla.cho_solve(self._chol, np.eye(k))
        else:
            inner = self._pinv
        X[np.ix_(self.live, self.live)] = inner
        return X

    def project(self, v: np.ndarray) -> np.ndarray:
        """proj_{range B^T}(v) = B^T (B B^T)^+ B v."""
        v = np.asarray(v, dtype=np.float64)
        w = self.solve_normal(self.B @ v, x0=getattr(self, "_warm", None))
        if self.method == "pcg":
            self._warm = w
        return self.B.T @ w

    def reflect(self, v: np.ndarray) -> np.ndarray:
        """abs_{range B^T}(v) = 2 proj(v) - v (Def. 1 for a subspace)."""
        return 2.0 * self.project(v) - np.asarray(v, dtype=np.float64)

    def pinv_apply(self, b: np.ndarray) -> np.ndarray:
        """B^dagger b = B^T (B B^T)^+ b."""
        return self.B.T @ self.solve_normal(b)
