"""Comparison helpers of the GPU parity tests.

Every vector comparison is made two ways: normwise, ||g - ref|| / ||ref||,
and element by element, max_i |g_i - ref_i| / max_i |ref_i|.  A normwise bar
alone would let a few entries of a long vector drift far beyond it."""
import numpy as np


def rel(a, b) -> float:
    """||a - b||_2 / ||b||_2."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def elem(a, b) -> float:
    """max_i |a_i - b_i| / max_i |b_i|."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) if b.size else 0.0


def errors(g: dict, ref: dict, keys) -> dict:
    return {k: (rel(g[k], ref[k]), elem(g[k], ref[k])) for k in keys}


def fmt(errs: dict) -> str:
    return " ".join(f"{k} {n:.2e}/{e:.2e}" for k, (n, e) in errs.items())


def assert_close(errs: dict, tol: float, tags=""):
    """Both measures of every key within tol."""
    for k, (n, e) in errs.items():
        assert n <= tol, f"{tags} {k}: normwise {n:.3e} > {tol:.1e}"
        assert e <= tol, f"{tags} {k}: elementwise {e:.3e} > {tol:.1e}"


def obj_err(pobj: float, p_star: float) -> float:
    return abs(pobj - p_star) / (1.0 + abs(p_star))
