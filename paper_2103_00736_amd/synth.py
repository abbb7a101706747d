"""Seeded synthetic conic problems (LP and SOCP) with a planted optimum.

This module only draws inputs: random sparsity patterns, values and a
primal/dual pair that is optimal by construction.  It holds none of the
solver's arithmetic, so both the CPU checker and the GPU solver can consume
the same instances.

Problem form (the primal of Section II, eq. prob_primal):
    minimise c^T x  subject to  A x = b,  x in K,
with K = R_+^{n_orth} x L_{k_1} x ... x L_{k_r}: an orthant block first,
then the Lorentz cones in list order (an orthant coordinate is a Lorentz
cone of size one).  The dual is  maximise b^T y  s.t.  A^T y + z = c, z in K.

Planting: pick x0 in K, z0 in K with x0^T z0 = 0, any y0, then set
b = A x0 and c = A^T y0 + z0.  (x0, y0, z0) then satisfies the KKT system,
so p* = c^T x0 = b^T y0 exactly.  All matrix values are rounded to float32
before planting, so a float32 copy of A is exactly the problem's A.

Seeds: instance seed = 20210301 + config * 1_000_000 + index.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Iterator, List, Optional

import numpy as np

BASE_SEED = 20210301


def instance_seed(config: int, index: int = 0) -> int:
    return BASE_SEED + config * 1_000_000 + index


@dataclasses.dataclass
class ConicProblem:
    """CSR matrix A (m x n), vectors b (m), c (n) and a cone list."""

    m: int
    n: int
    row_ptr: np.ndarray  # int64, m+1
    col_idx: np.ndarray  # int32, nnz (ascending within a row)
    val: np.ndarray  # float64, nnz (float32-representable)
    b: np.ndarray  # float64, m
    c: np.ndarray  # float64, n
    n_orth: int
    soc_sizes: np.ndarray  # int32, sizes of the Lorentz cones after the orthant block
    x0: Optional[np.ndarray] = None  # planted primal optimum
    y0: Optional[np.ndarray] = None  # planted dual multiplier
    z0: Optional[np.ndarray] = None  # planted dual slack
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def p_star(self) -> float:
        return float(self.c @ self.x0)

    @property
    def is_socp(self) -> bool:
        return len(self.soc_sizes) > 0

    def scipy_csr(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.m, self.n))

    def nbytes_device(self, value_bytes: int = 4) -> int:
        """Rough device footprint: CSR of A and of A^T plus ~16 vectors."""
        nnz = self.nnz
        return 2 * nnz * (value_bytes + 4) * 2 + 4 * (self.m + self.n) + 16 * value_bytes * (self.m + self.n)


# ----------------------------------------------------------------------------
# sparsity patterns
# ----------------------------------------------------------------------------

def _csr_from_cols(m: int, n: int, rows_per_col: np.ndarray) -> tuple:
    """rows_per_col: (n, k) distinct row indices per column -> CSR (row_ptr, col_idx, order)."""
    k = rows_per_col.shape[1]
    rows = rows_per_col.reshape(-1)
    cols = np.repeat(np.arange(n, dtype=np.int64), k)
    order = np.argsort(rows, kind="stable")  # stable: columns stay ascending within a row
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, cols[order].astype(np.int32), order


def _distinct_rows(rng: np.random.Generator, m: int, n: int, k: int, cdf: Optional[np.ndarray]) -> np.ndarray:
    """k distinct rows for each of n columns, uniform or by the given CDF."""
    if k > m:
        raise ValueError("more nonzeros per column than rows")

    def draw(cnt):
        if cdf is None:
            return rng.integers(0, m, size=(cnt, k), dtype=np.int64)
        r = np.searchsorted(cdf, rng.random((cnt, k)), side="right")
        return np.minimum(r, m - 1).astype(np.int64)

    rows = draw(n)
    while True:
        srt = np.sort(rows, axis=1)
        dup = np.nonzero((srt[:, 1:] == srt[:, :-1]).any(axis=1))[0]
        if dup.size == 0:
            return rows
        rows[dup] = draw(dup.size)


def _uniform_positions(rng: np.random.Generator, m: int, n: int, nnz: int) -> tuple:
    """Exactly nnz distinct positions uniform in the m x n grid -> CSR pattern."""
    flat = np.sort(rng.choice(m * n, size=nnz, replace=False))
    rows = flat // n
    cols = (flat % n).astype(np.int32)
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, cols


def _f32(a: np.ndarray) -> np.ndarray:
    return np.asarray(a, dtype=np.float32).astype(np.float64)


# ----------------------------------------------------------------------------
# planted optimum
# ----------------------------------------------------------------------------

def _plant_orthant(rng: np.random.Generator, n: int) -> tuple:
    """Half of the coordinates carry x0 ~ U(0,1), the others z0 ~ U(0,1)."""
    x0 = np.zeros(n)
    z0 = np.zeros(n)
    support = rng.permutation(n)[: n // 2]
    mask = np.zeros(n, dtype=bool)
    mask[support] = True
    x0[mask] = _f32(rng.random(mask.sum()))
    z0[~mask] = _f32(rng.random((~mask).sum()))
    return x0, z0


def _plant_soc(rng: np.random.Generator, k: int) -> tuple:
    """One Lorentz cone of size k: (x interior, z=0), (x=0, z interior) or
    both on the boundary with x^T z = 0, each with probability 1/3."""
    u = _f32(rng.standard_normal(k - 1) / math.sqrt(max(k - 1, 1)))
    nu = float(np.linalg.norm(u))
    x = np.zeros(k)
    z = np.zeros(k)
    kind = rng.integers(0, 3)
    if kind == 0:
        x[0] = nu + 0.1 + 0.9 * rng.random()
        x[1:] = u
    elif kind == 1:
        z[0] = nu + 0.1 + 0.9 * rng.random()
        z[1:] = u
    else:
        beta = 0.5 + 1.5 * rng.random()
        x[0] = nu
        x[1:] = u
        z[0] = beta * nu
        z[1:] = -beta * u
    return x, z


def _finish(rng, m, n, row_ptr, col_idx, val, x0, z0, n_orth, soc_sizes, name) -> ConicProblem:
    import scipy.sparse as sp

    y0 = _f32(rng.standard_normal(m))
    A = sp.csr_matrix((val, col_idx, row_ptr), shape=(m, n))
    b = A @ x0
    c = A.T @ y0 + z0
    return ConicProblem(m=m, n=n, row_ptr=row_ptr.astype(np.int64), col_idx=col_idx.astype(np.int32),
                        val=val, b=np.asarray(b, dtype=np.float64), c=np.asarray(c, dtype=np.float64),
                        n_orth=int(n_orth), soc_sizes=np.asarray(soc_sizes, dtype=np.int32),
                        x0=x0, y0=y0, z0=z0, name=name)


@dataclasses.dataclass
class DenseProblem:
    """Dense A (m x n, row-major float64 holding float32 values), b, c and a
    cone list (orthant block first, then Lorentz cones); no planted optimum."""

    m: int
    n: int
    A: np.ndarray
    b: np.ndarray
    c: np.ndarray
    n_orth: int
    soc_sizes: np.ndarray
    x_feas: Optional[np.ndarray] = None  # the cone point b was built from
    name: str = ""

    @property
    def nnz(self) -> int:
        return self.m * self.n

    @property
    def is_socp(self) -> bool:
        return len(self.soc_sizes) > 0

    def scipy_csr(self):
        import scipy.sparse as sp

        return sp.csr_matrix(self.A)


# ----------------------------------------------------------------------------
# generators
# ----------------------------------------------------------------------------

def lp_uniform(m: int, n: int, nnz: int, seed: int, name: str = "lp_uniform") -> ConicProblem:
    """Exactly nnz positions uniform without replacement, N(0,1) values, K = R_+^n."""
    rng = np.random.default_rng(seed)
    nnz = max(1, min(int(nnz), m * n))
    row_ptr, col_idx = _uniform_positions(rng, m, n, nnz)
    val = _f32(rng.standard_normal(nnz))
    x0, z0 = _plant_orthant(rng, n)
    return _finish(rng, m, n, row_ptr, col_idx, val, x0, z0, n, [], name)


def lp_powerlaw(m: int, n: int, per_col: int, seed: int, exponent: float = 2.5,
                row_scale_decades: float = 3.0, name: str = "lp_powerlaw") -> ConicProblem:
    """Chung-Lu pattern: row weights w_i = (1-U)^(-1/(exponent-1)) give a degree
    law ~ w^-exponent; each column takes per_col distinct rows with P ~ w.
    N(0,1) values; row i scaled by 10^U(-d, d)."""
    rng = np.random.default_rng(seed)
    w = (1.0 - rng.random(m)) ** (-1.0 / (exponent - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    rows = _distinct_rows(rng, m, n, per_col, cdf)
    row_ptr, col_idx, order = _csr_from_cols(m, n, rows)
    vals_colmajor = rng.standard_normal(n * per_col)
    scale = 10.0 ** rng.uniform(-row_scale_decades, row_scale_decades, size=m)
    row_of = np.repeat(np.arange(m), np.diff(row_ptr))
    val = _f32(vals_colmajor[order] * scale[row_of])
    x0, z0 = _plant_orthant(rng, n)
    return _finish(rng, m, n, row_ptr, col_idx, val, x0, z0, n, [], name)


def lp_percol(m: int, n: int, per_col: int, seed: int, name: str = "lp_percol") -> ConicProblem:
    """per_col distinct uniform rows in every column, N(0,1) values, K = R_+^n."""
    rng = np.random.default_rng(seed)
    rows = _distinct_rows(rng, m, n, per_col, None)
    row_ptr, col_idx, order = _csr_from_cols(m, n, rows)
    val = _f32(rng.standard_normal(n * per_col)[order])
    x0, z0 = _plant_orthant(rng, n)
    return _finish(rng, m, n, row_ptr, col_idx, val, x0, z0, n, [], name)


def soc_sizes_fill(rng: np.random.Generator, n: int, lo: int, hi: int, fill: float) -> np.ndarray:
    """Cone sizes uniform in {lo..hi}, drawn until the next one would push the
    SOC part past fill*n."""
    cap = int(fill * n)
    sizes: List[int] = []
    total = 0
    while True:
        k = int(rng.integers(lo, hi + 1))
        if total + k > cap:
            break
        sizes.append(k)
        total += k
    return np.asarray(sizes, dtype=np.int32)


def socp_percol(m: int, n: int, per_col: int, seed: int, soc_lo: int = 3, soc_hi: int = 50,
                soc_fill: float = 0.9, name: str = "socp_percol") -> ConicProblem:
    """SOCP: Lorentz cones of sizes U{soc_lo..soc_hi} fill soc_fill*n, the rest
    is an orthant block placed first; per_col distinct uniform rows per column."""
    rng = np.random.default_rng(seed)
    sizes = soc_sizes_fill(rng, n, soc_lo, soc_hi, soc_fill)
    n_orth = n - int(sizes.sum())
    rows = _distinct_rows(rng, m, n, per_col, None)
    row_ptr, col_idx, order = _csr_from_cols(m, n, rows)
    val = _f32(rng.standard_normal(n * per_col)[order])
    x0 = np.zeros(n)
    z0 = np.zeros(n)
    x0[:n_orth], z0[:n_orth] = _plant_orthant(rng, n_orth)
    off = n_orth
    for k in sizes:
        x0[off:off + k], z0[off:off + k] = _plant_soc(rng, int(k))
        off += k
    return _finish(rng, m, n, row_ptr, col_idx, val, x0, z0, n_orth, sizes, name)


# ----------------------------------------------------------------------------
# the five workload configurations
# ----------------------------------------------------------------------------

def config0(index: int = 0) -> ConicProblem:
    """LP 200 x 500, exactly 2% density (2000 nonzeros), N(0,1), K = R_+^500."""
    return lp_uniform(200, 500, 2000, instance_seed(0, index), name="cfg0_lp_200x500")


def config1(index: int = 0, scale: float = 1.0) -> ConicProblem:
    """LP m=500k, n=2M, 5 nonzeros per column, power-law row degrees (exponent
    2.5), row scales 10^U(-3,3).  `scale` shrinks m and n for tests."""
    m = max(8, int(500_000 * scale))
    n = max(16, int(2_000_000 * scale))
    return lp_powerlaw(m, n, 5, instance_seed(1, index), name=f"cfg1_lp_{m}x{n}")


def config2(index: int = 0, scale: float = 1.0) -> ConicProblem:
    """SOCP n=1M (Lorentz cones U{3..50} filling 0.9 n, orthant remainder),
    m=300k, 8 nonzeros per column."""
    m = max(16, int(300_000 * scale))
    n = max(64, int(1_000_000 * scale))
    return socp_percol(m, n, 8, instance_seed(2, index), 3, 50, 0.9, name=f"cfg2_socp_{m}x{n}")


def config3_sizes(count: int = 4096) -> np.ndarray:
    rng = np.random.default_rng(instance_seed(3, 999_999))
    return rng.integers(50, 2001, size=count)


def config3(index: int, m: Optional[int] = None) -> ConicProblem:
    """One small LP of the 4096-instance batch: m ~ U{50..2000}, n = 2.5 m,
    exactly round(0.01 m n) uniform positions, N(0,1)."""
    if m is None:
        m = int(config3_sizes(max(4096, index + 1))[index])
    n = int(2.5 * m)
    nnz = max(1, int(round(0.01 * m * n)))
    return lp_uniform(m, n, nnz, instance_seed(3, index), name=f"cfg3_lp_{m}x{n}")


@dataclasses.dataclass
class Request:
    index: int
    arrival_s: float
    kind: str  # "lp" or "socp"
    m: int

    def problem(self) -> ConicProblem:
        seed = instance_seed(4, self.index)
        n = 3 * self.m
        if self.kind == "lp":
            return lp_percol(self.m, n, 6, seed, name=f"cfg4_lp_{self.m}")
        return socp_percol(self.m, n, 6, seed, 3, 30, 1.0, name=f"cfg4_socp_{self.m}")


def config4_trace(count: int = 2000, rate_per_s: float = 200.0, m_lo: float = 1e3,
                  m_hi: float = 2e5) -> List[Request]:
    """Poisson arrivals (exponential gaps, mean 1/rate), 70% LP / 30% SOCP,
    m log-uniform in [m_lo, m_hi], n = 3m, 6 nonzeros per column."""
    rng = np.random.default_rng(instance_seed(4, 999_999))
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    kinds = np.where(rng.random(count) < 0.7, "lp", "socp")
    ms = np.rint(np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), size=count))).astype(int)
    return [Request(i, float(t[i]), str(kinds[i]), int(ms[i])) for i in range(count)]


def synthetic_state(p, seed: int, spread: float) -> tuple:
    """A seeded state (s_prev, s, O, w) for one-iteration tests of a problem:
    s and s_prev ~ N(0,1) rounded to FP32, O = exp(U(-spread/2, spread/2)) drawn
    once per cone (an orthant coordinate is a cone of one) so that it is
    constant on every cone, w ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    s = _f32(rng.standard_normal(p.n))
    s_prev = _f32(rng.standard_normal(p.n))
    sizes = np.concatenate([np.ones(p.n_orth, dtype=np.int64), np.asarray(p.soc_sizes, dtype=np.int64)])
    O = np.repeat(np.exp(rng.uniform(-spread / 2, spread / 2, size=sizes.size)), sizes)
    w = rng.standard_normal(p.m)
    return s_prev, s, O, w


def iter_batch(count: int) -> Iterator[ConicProblem]:
    for i in range(count):
        yield config3(i)


# ----------------------------------------------------------------------------
# the paper's dense instances (Sec. V-B linear programs, Sec. V-D SOCPs)
# ----------------------------------------------------------------------------

def e3_lp(n: int, index: int = 0) -> DenseProblem:
    """Dense LP of the paper's LP study: m = floor(0.8 n), A ~ U[-1, 1], b = A x
    with x half-normal (absolute values of N(0,1) draws), c ~ N(0,1),
    K = R_+^n.  Values rounded to float32."""
    rng = np.random.default_rng(instance_seed(5, index) + n)
    m = int(0.8 * n)
    A = _f32(rng.uniform(-1.0, 1.0, size=(m, n)))
    x = np.abs(rng.standard_normal(n))
    c = _f32(rng.standard_normal(n))
    return DenseProblem(m=m, n=n, A=A, b=A @ x, c=c, n_orth=n, soc_sizes=np.zeros(0, np.int32), x_feas=x,
                        name=f"e3_lp_{m}x{n}")


def e6_socp(n: int, h: int, index: int = 0) -> DenseProblem:
    """Dense SOCP of the paper's SOCP study: m = floor(0.8 n), A ~ U[-1, 1],
    c ~ U[0, 1], K = Lorentz cones of size h (an orthant block takes n mod h
    coordinates).  b = A x with x drawn strictly inside K: per cone the tail
    u ~ U[0,1]^(h-1) and the head ||u|| + U(0,1); orthant coordinates U(0,1).
    Values rounded to float32."""
    rng = np.random.default_rng(instance_seed(6, index) + 100 * n + h)
    m = int(0.8 * n)
    n_orth = n % h
    sizes = np.full((n - n_orth) // h, h, dtype=np.int32)
    A = _f32(rng.uniform(-1.0, 1.0, size=(m, n)))
    x = np.empty(n)
    x[:n_orth] = rng.random(n_orth)
    for k in range(len(sizes)):
        off = n_orth + k * h
        u = rng.random(h - 1)
        x[off + 1:off + h] = u
        x[off] = np.sqrt(u @ u) + rng.random()
    c = _f32(rng.random(n))
    return DenseProblem(m=m, n=n, A=A, b=A @ x, c=c, n_orth=n_orth, soc_sizes=sizes, x_feas=x,
                        name=f"e6_socp_h{h}_{m}x{n}")


def e2_lp(index: int) -> DenseProblem:
    """One of the 10 random LPs of the paper's conditioning-schedule example
    (Sec. IV): A in R^{80x100} with N(0,1) entries, b = A x with x ~ U[0,1]^100,
    c ~ N(0,1), K = R_+^100.  Values rounded to float32."""
    rng = np.random.default_rng(instance_seed(7, index))
    A = _f32(rng.standard_normal((80, 100)))
    x = rng.random(100)
    c = _f32(rng.standard_normal(100))
    return DenseProblem(m=80, n=100, A=A, b=A @ x, c=c, n_orth=100, soc_sizes=np.zeros(0, np.int32), x_feas=x,
                        name=f"e2_lp_{index}")
