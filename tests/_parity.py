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


def assert_close(errs: dict, tol: float, tags="", elem_tol=None, norm_only=()):
    """Normwise error of every key within tol; elementwise within elem_tol
    (default tol), except for the keys in norm_only."""
    et = tol if elem_tol is None else elem_tol
    for k, (n, e) in errs.items():
        assert n <= tol, f"{tags} {k}: normwise {n:.3e} > {tol:.1e}"
        if k not in norm_only:
            assert e <= et, f"{tags} {k}: elementwise {e:.3e} > {et:.1e}"


# Bars of the one-iteration parity tests.  Mixed precision: 1e-5 relative
# (the FP32 bar), normwise and element by element.  FP64: 1e-9 normwise; the
# CG stops at 1e-13 of its initial residual, which bounds the error of the
# projection in norm only, and element by element the measured errors run up
# to about ten times the normwise ones, so the elementwise FP64 bar is 1e-8.
# x = O (p + s+)/2 is compared normwise and, element by element, in the scaled
# space of the iteration (x / O = (p + s+)/2): after a conditioning event O
# spans up to e^t, and x_j carries O_j times the error of the scaled iterate.
TOL_MIXED = 1e-5
TOL_FP64 = 1e-9
TOL_FP64_ELEM = 1e-8


def iterate_errors(g: dict, ref: dict, O, keys=("s", "x", "z", "y")) -> dict:
    """errors() of the iterate, with x/O added beside x when x is compared."""
    g, ref = dict(g), dict(ref)
    keys = list(keys)
    if "x" in keys:
        g["x/O"] = np.asarray(g["x"]) / np.asarray(O)
        ref["x/O"] = np.asarray(ref["x"]) / np.asarray(O)
        keys.insert(keys.index("x") + 1, "x/O")
    return errors(g, ref, keys)


def assert_iterate(errs: dict, fp64: bool, tags=""):
    """The one-iteration bars above (x normwise only; x/O both ways)."""
    if fp64:
        assert_close(errs, TOL_FP64, tags, elem_tol=TOL_FP64_ELEM, norm_only=("x",))
    else:
        assert_close(errs, TOL_MIXED, tags, norm_only=("x",))


def obj_err(pobj: float, p_star: float) -> float:
    return abs(pobj - p_star) / (1.0 + abs(p_star))
