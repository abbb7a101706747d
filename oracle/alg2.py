"""Algorithm 2 (adaptive conditioning) of the paper, step by step, in FP64.

Test infrastructure only (see the package header).

Algorithm 2 keeps a diagonal positive scaling O (constant inside every cone),
works on the scaled problem  min (O c)^T x_hat,  (A O) x_hat = b,  x_hat in
O^{-1} K  (Sec. IV; x_hat = O^{-1} x, z_hat = O z), and iterates

    p <- abs_{O^{-1}K}(s)                       (step 16)
    r <- abs_{A_hat}(p),  A_hat = range((AO)^T) (step 17)
    s <- s/2 - r/2 + d                          (step 18)
    x <- O (p + s) / 2                          (step 19)
    z <- O^{-1} (p - s) / (2 mu)                (step 20)

and at the iterations l in L u {1} it recomputes O from the current x and z
(steps 5-11), rebuilds A_hat and d (steps 12-13) and re-expresses s in the
new scaling (step 14).  Algorithm 1 is the same loop with L empty: at l = 1
the conditioning of x = z = e_K gives O = I.

Readings of the paper taken here (the same ones the GPU solver follows):
  * Initial point: x = z = e_K (1 on orthant coordinates, (1,0,..,0) on each
    Lorentz block).  The Require line only asks for z with no zero entries.
  * t: any t > 0 (the Require line says 0 < t < 1, but every experiment uses
    t = 9.2 or 1.7).  log is the natural logarithm; the power in step 11 is
    elementwise, so log(max O) - log(min O) = min(t, log(max o) - log(min o)).
  * Steps 5-10 divide by |z_{h+1}|, which can vanish, and the numerator can
    vanish too.  Guard: 0/0 counts as 1; then the log range is taken over the
    finite positive ratios, a zero ratio is replaced by their minimum and an
    infinite one by their maximum; with no finite positive ratio, O = I.
  * abs_{O^{-1}K} = abs_K because O is a positive constant on every cone and
    cones are invariant under positive scaling (checked by an assertion).
  * x and z of steps 19-20 use p of the current iteration and the updated s
    (the listing's order); those are the x, z the next conditioning reads.
  * Dual multiplier: y_w = -w / mu with (A O^2 A^T) w = A O (p - mu O c) - b,
    the multiplier of the scaled dual ((AO)^T y + z_hat = O c, Sec. IV), which
    at a fixed point s+ = s satisfies A^T y + z = c.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np
import scipy.sparse as sp

from .cones import abs_K, blocks, e_K
from .kkt import kkt_errors
from .subspace import RangeProjector


@dataclasses.dataclass(frozen=True)
class Schedule:
    """The set L of conditioning iterations, as {first, first+every, ...} up to
    `last` (inclusive, -1 = unbounded).  first = 0 means L is empty; every = 0
    means L = {first}.  Iteration 1 always conditions (Alg. 2 step 4)."""

    first: int = 300
    every: int = 100
    last: int = -1

    def __contains__(self, l: int) -> bool:
        if l == 1:
            return True
        if self.first <= 0 or l < self.first:
            return False
        if self.last >= 0 and l > self.last:
            return False
        if self.every <= 0:
            return l == self.first
        return (l - self.first) % self.every == 0


LP_SCHEDULE = Schedule(300, 100, -1)  # Sec. V-A: L = {300, 400, ...}, t = 9.2, mu = 1
SOCP_SCHEDULE = Schedule(200, 100, -1)  # Sec. V-C: L = {200, 300, ...}, t = 1.7, mu = 1
LP_T = 9.2
SOCP_T = 1.7
NO_CONDITIONING = Schedule(0, 0, -1)


def conditioning_ratio(x: np.ndarray, z: np.ndarray, n_orth: int, soc_sizes: Sequence[int]) -> np.ndarray:
    """Steps 5-10: for the cone occupying [h+1, h+n_i] (1-based), every entry j
    of the block gets o_j = |x_{h+1} - ||x_{h+2..h+n_i}||_2| / |z_{h+1}|.
    Returns the raw ratio (may contain 0, inf or nan for 0/0)."""
    o = np.empty_like(np.asarray(x, dtype=np.float64))
    with np.errstate(divide="ignore", invalid="ignore"):
        for start, k in blocks(n_orth, soc_sizes):
            num = abs(x[start] - np.linalg.norm(x[start + 1:start + k]))
            den = abs(z[start])
            o[start:start + k] = num / den
    return o


def normalize_scaling(o_raw: np.ndarray, t: float) -> np.ndarray:
    """Step 11: O = diag(|o|)^min(1, t / (log max o - log min o)), with the
    guard for zero / infinite / undefined ratios described in the module."""
    o = np.abs(np.asarray(o_raw, dtype=np.float64))
    o = np.where(np.isnan(o), 1.0, o)  # 0/0
    valid = np.isfinite(o) & (o > 0)
    if not valid.any():
        return np.ones_like(o)
    lo = o[valid].min()
    hi = o[valid].max()
    o = np.where(o == 0, lo, o)
    o = np.where(np.isinf(o), hi, o)
    span = np.log(hi) - np.log(lo)
    alpha = 1.0 if span <= 0 else min(1.0, t / span)
    return o ** alpha


class Algorithm2:
    """State and steps of Algorithm 2 for one problem (A, b, c, K)."""

    def __init__(self, A, b, c, n_orth: int, soc_sizes: Sequence[int], mu: float = 1.0,
                 t: float = LP_T, schedule: Schedule = LP_SCHEDULE, method: str = "auto"):
        self.A = sp.csr_matrix(A, dtype=np.float64)
        self.b = np.asarray(b, dtype=np.float64)
        self.c = np.asarray(c, dtype=np.float64)
        self.m, self.n = self.A.shape
        self.n_orth = int(n_orth)
        self.soc_sizes = [int(k) for k in soc_sizes]
        if self.n_orth + sum(self.soc_sizes) != self.n:
            raise ValueError("cone sizes do not add up to n")
        self.mu = float(mu)
        self.t = float(t)
        self.schedule = schedule
        self.method = method
        # Require line: initial x and z (reading: x = z = e_K)
        self.x = e_K(self.n_orth, self.soc_sizes)
        self.z = e_K(self.n_orth, self.soc_sizes)
        self.l = 0  # step 1
        self.O = np.ones(self.n)
        self.s = np.zeros(self.n)
        self.p = np.zeros(self.n)
        self.d = None
        self.proj: Optional[RangeProjector] = None

    # -- steps 5-14 ------------------------------------------------------------
    def condition(self) -> None:
        o = conditioning_ratio(self.x, self.z, self.n_orth, self.soc_sizes)  # steps 5-10
        O = normalize_scaling(o, self.t)  # step 11
        self._check_blockwise_constant(O)
        self.O = O
        self.proj = RangeProjector(self.A, O, method=self.method)  # step 12
        Oc = O * self.c
        self.d = self.proj.pinv_apply(self.b) + 0.5 * self.mu * (self.proj.reflect(Oc) - Oc)  # step 13
        self.s = self.x / O - self.mu * O * self.z  # step 14

    def _check_blockwise_constant(self, O: np.ndarray) -> None:
        for start, k in blocks(self.n_orth, self.soc_sizes):
            if k > 1 and not np.all(O[start:start + k] == O[start]):
                raise AssertionError("O must be constant inside every cone")

    # -- one pass of the repeat loop (steps 3-20) ------------------------------
    def step(self) -> None:
        self.l += 1  # step 3
        if self.l in self.schedule:  # step 4
            self.condition()
        s = self.s
        p = abs_K(s, self.n_orth, self.soc_sizes)  # step 16
        r = self.proj.reflect(p)  # step 17
        s_new = 0.5 * s - 0.5 * r + self.d  # step 18
        self.x = self.O * (p + s_new) / 2.0  # step 19
        self.z = (p - s_new) / (2.0 * self.mu * self.O)  # step 20
        self.p = p
        self.s = s_new

    def dual_multiplier(self) -> np.ndarray:
        """y_w = -w/mu with (A O^2 A^T) w = A O (p - mu O c) - b (p of the last step)."""
        B = self.proj.B
        w = self.proj.solve_normal(B @ (self.p - self.mu * self.O * self.c) - self.b)
        return -w / self.mu

    def kkt(self) -> Dict[str, float]:
        return kkt_errors(self.A, self.b, self.c, self.n_orth, self.soc_sizes, self.x, self.dual_multiplier(), self.z)

    def run(self, max_iter: int, eps: float = 0.0, check_every: int = 10,
            callback: Optional[Callable[["Algorithm2"], None]] = None, obj_stop: float = 0.0) -> Dict[str, float]:
        """Iterate until kkt <= eps at a check (every `check_every` iterations),
        and also obj_stop * eps_obj <= eps when obj_stop > 0, or max_iter
        iterations; returns the last KKT record (with 'iters')."""
        rec: Dict[str, float] = {}
        while self.l < max_iter:
            self.step()
            if callback is not None:
                callback(self)
            if eps > 0 and (self.l % check_every == 0 or self.l == max_iter):
                rec = self.kkt()
                if rec["kkt"] <= eps and obj_stop * rec["eps_obj"] <= eps:
                    break
        if not rec or rec.get("iters") != self.l:
            rec = self.kkt()
        rec["iters"] = self.l
        return rec


def default_parameters(soc_sizes: Sequence[int]):
    """(t, schedule) per problem class: LP t=9.2, L={300,400,..}; SOCP t=1.7,
    L={200,300,..} (Sec. V-A and V-C); mu = 1 in both."""
    if len(soc_sizes) > 0:
        return SOCP_T, SOCP_SCHEDULE
    return LP_T, LP_SCHEDULE


def one_iteration(A, b, c, n_orth: int, soc_sizes: Sequence[int], mu: float, s: np.ndarray,
                  O: np.ndarray, method: str = "auto") -> Dict[str, np.ndarray]:
    """One pass of steps 16-20 from a given (s, O), with d and A_hat of steps
    12-13 built for that O.  Returns p, s_next, x, z and y_w."""
    alg = Algorithm2(A, b, c, n_orth, soc_sizes, mu=mu, t=1.0, schedule=NO_CONDITIONING, method=method)
    alg.O = np.asarray(O, dtype=np.float64)
    alg._check_blockwise_constant(alg.O)
    alg.proj = RangeProjector(alg.A, alg.O, method=method)
    Oc = alg.O * alg.c
    alg.d = alg.proj.pinv_apply(alg.b) + 0.5 * mu * (alg.proj.reflect(Oc) - Oc)
    alg.s = np.asarray(s, dtype=np.float64).copy()
    alg.l = 1  # so that step() does not condition
    alg.step()
    return {"p": alg.p, "s": alg.s, "x": alg.x, "z": alg.z, "y": alg.dual_multiplier(), "d": alg.d}


def run_history(alg: Algorithm2, iters: int) -> List[np.ndarray]:
    """The iterates s^1..s^iters (for invariants of Lemma 3)."""
    out = []
    for _ in range(iters):
        alg.step()
        out.append(alg.s.copy())
    return out
