"""ctypes binding of libacs.so (include/acs.h): argument marshalling only.

Every step of the solver runs in the library's HIP kernels.  If the shared
library is missing this module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libacs.so")

ACS_OK = 0
ACS_PENDING = 1
ACS_ERR_ARG = -1
ACS_ERR_NOMEM = -2
ACS_ERR_DEVICE = -3
ACS_ERR_NUMERIC = -4
ACS_ERR_STATE = -5

SOLVED, MAX_ITER, NUMERIC, CANCELLED = 0, 1, 2, 3
PREC_MIXED, PREC_FP64 = 0, 1
PROJ_CG, PROJ_FACTOR, PROJ_AUTO = 0, 1, 2

# timing classes of acs_state_timing
(KC_UPDATE, KC_RESID, KC_CG_T, KC_CG_A, KC_CONE, KC_CHECK, KC_COND, KC_FIN, KC_CG_COMB, KC_FAC_SYRK, KC_FAC_UPDATE,
 KC_FAC_APPLY, KC_FAC_PANEL) = range(13)
PROF_ALL = (1 << 13) - 1  # ACS_PROF_ALL

EXPORTED = [
    "acs_version", "acs_last_error", "acs_init", "acs_settings_default", "acs_problem_create",
    "acs_problem_destroy", "acs_problem_create_dense", "acs_problem_device_bytes", "acs_problem_factor_bytes",
    "acs_batch_device_bytes", "acs_solve", "acs_solve_device", "acs_solve_device_noalloc", "acs_state_create", "acs_state_destroy",
    "acs_state_set", "acs_state_step", "acs_state_solve", "acs_state_get", "acs_state_info", "acs_state_check",
    "acs_state_spmv", "acs_state_profile", "acs_state_timing", "acs_state_normal_inverse", "acs_batch_create", "acs_batch_destroy",
    "acs_batch_autotune", "acs_batch_run", "acs_batch_result", "acs_batch_state_get", "acs_batch_lanes",
    "acs_batch_solve",
    "acs_server_create", "acs_server_destroy", "acs_server_submit", "acs_server_poll", "acs_server_wait",
    "acs_server_cancel", "acs_server_stats",
]


class AcsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"acs error {code}: {msg}")
        self.code = code


class Settings(ctypes.Structure):
    _fields_ = [
        ("mu", ctypes.c_double), ("t", ctypes.c_double),
        ("l_first", ctypes.c_int32), ("l_every", ctypes.c_int32), ("l_last", ctypes.c_int32),
        ("auto_params", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
        ("eps_kkt", ctypes.c_double), ("precision", ctypes.c_int32), ("cg_max", ctypes.c_int32),
        ("cg_reduce", ctypes.c_double), ("cg_abs", ctypes.c_double), ("verbose", ctypes.c_int32),
        ("projection", ctypes.c_int32), ("obj_stop", ctypes.c_int32), ("equilibrate", ctypes.c_int32),
        ("eq_sweeps", ctypes.c_int32), ("a_slices", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("iterations", ctypes.c_int32), ("cg_steps", ctypes.c_int64),
        ("conditionings", ctypes.c_int32), ("reserved0", ctypes.c_int32),
        ("eps_p", ctypes.c_double), ("eps_d", ctypes.c_double), ("eps_gap", ctypes.c_double),
        ("eps_cone", ctypes.c_double), ("kkt", ctypes.c_double), ("pobj", ctypes.c_double),
        ("dobj", ctypes.c_double), ("solve_ms", ctypes.c_double), ("setup_ms", ctypes.c_double),
        ("alpha", ctypes.c_double), ("o_range", ctypes.c_double), ("queue_ms", ctypes.c_double),
        ("latency_ms", ctypes.c_double), ("eps_obj", ctypes.c_double), ("reserved", ctypes.c_double * 3),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("reserved")}


class ServerStats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int64), ("running", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_int64), ("ticks", ctypes.c_int64), ("peak_running", ctypes.c_int64),
                ("reserved", ctypes.c_int64 * 2)]


_lib = None
P = ctypes.c_void_p
DP = ctypes.POINTER(ctypes.c_double)
I32P = ctypes.POINTER(ctypes.c_int32)
I64P = ctypes.POINTER(ctypes.c_int64)


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_00736_amd.build`")
    # One HIP runtime per process: when torch is installed, load it first so
    # that libacs binds to the HIP runtime torch already holds (same soname)
    # and torch-allocated device buffers and streams are valid in libacs.  A
    # second runtime loaded beside an initialised one leaves torch without a
    # device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "acs_version": (ctypes.c_char_p, []),
        "acs_last_error": (ctypes.c_char_p, []),
        "acs_init": (ctypes.c_int, [ctypes.c_int32]),
        "acs_settings_default": (None, [ctypes.POINTER(Settings)]),
        "acs_problem_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, I64P, I32P, DP, DP, DP,
                                              ctypes.c_int32, ctypes.c_int32, I32P, ctypes.POINTER(P)]),
        "acs_problem_destroy": (None, [P]),
        "acs_problem_create_dense": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, DP, DP, DP, ctypes.c_int32,
                                                    ctypes.c_int32, I32P, ctypes.POINTER(P)]),
        "acs_problem_device_bytes": (ctypes.c_int64, [P, ctypes.c_int32]),
        "acs_problem_factor_bytes": (ctypes.c_int64, [P]),
        "acs_batch_device_bytes": (ctypes.c_int64, [P]),
        "acs_solve": (ctypes.c_int, [P, ctypes.POINTER(Settings), DP, DP, DP, ctypes.POINTER(Info), P]),
        "acs_solve_device": (ctypes.c_int, [P, ctypes.POINTER(Settings), P, P, P, ctypes.POINTER(Info), P]),
        "acs_solve_device_noalloc": (ctypes.c_int, [P, ctypes.POINTER(Settings), P, P, P, ctypes.POINTER(Info), P]),
        "acs_state_create": (ctypes.c_int, [P, ctypes.POINTER(Settings), P, ctypes.POINTER(P)]),
        "acs_state_destroy": (None, [P]),
        "acs_state_set": (ctypes.c_int, [P, ctypes.c_int32, DP, DP, DP, DP]),
        "acs_state_step": (ctypes.c_int, [P, ctypes.c_int32]),
        "acs_state_solve": (ctypes.c_int, [P, ctypes.POINTER(Info)]),
        "acs_state_get": (ctypes.c_int, [P, I32P, DP, DP, DP, DP, DP, DP, DP]),
        "acs_state_info": (ctypes.c_int, [P, ctypes.POINTER(Info)]),
        "acs_state_check": (ctypes.c_int, [P, ctypes.POINTER(Info)]),
        "acs_state_spmv": (ctypes.c_int, [P, ctypes.c_int32, P, P, ctypes.c_int32, DP]),
        "acs_state_profile": (ctypes.c_int, [P, ctypes.c_int32]),
        "acs_state_timing": (ctypes.c_int, [P, ctypes.c_int32, I64P, DP]),
        "acs_state_normal_inverse": (ctypes.c_int, [P, DP]),
        "acs_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(Settings), P,
                                            ctypes.POINTER(P)]),
        "acs_batch_destroy": (None, [P]),
        "acs_batch_autotune": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p]),
        "acs_batch_run": (ctypes.c_int, [P, ctypes.c_int32, ctypes.c_int32, DP]),
        "acs_batch_result": (ctypes.c_int, [P, ctypes.c_int32, DP, DP, DP, ctypes.POINTER(Info)]),
        "acs_batch_lanes": (ctypes.c_int, [P, ctypes.c_int32, I32P, I32P]),
        "acs_batch_state_get": (ctypes.c_int, [P, ctypes.c_int32, I32P, DP, DP, DP, DP, DP]),
        "acs_batch_solve": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(Settings),
                                           ctypes.POINTER(DP), ctypes.POINTER(DP), ctypes.POINTER(DP),
                                           ctypes.POINTER(Info), P]),
        "acs_server_create": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.POINTER(P)]),
        "acs_server_destroy": (None, [P]),
        "acs_server_submit": (ctypes.c_int, [P, P, ctypes.POINTER(Settings), ctypes.POINTER(ctypes.c_uint64)]),
        "acs_server_poll": (ctypes.c_int, [P, ctypes.c_uint64, DP, DP, DP, ctypes.POINTER(Info)]),
        "acs_server_wait": (ctypes.c_int, [P, ctypes.c_uint64, ctypes.c_int32, DP, DP, DP, ctypes.POINTER(Info)]),
        "acs_server_cancel": (ctypes.c_int, [P, ctypes.c_uint64]),
        "acs_server_stats": (ctypes.c_int, [P, ctypes.POINTER(ServerStats)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int) -> int:
    if rc < 0:
        msg = lib().acs_last_error().decode(errors="replace")
        raise AcsError(rc, msg)
    return rc


def _dptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(DP)


def default_settings(**kw) -> Settings:
    s = Settings()
    lib().acs_settings_default(ctypes.byref(s))
    for k, v in kw.items():
        if not hasattr(s, k):
            raise KeyError(f"unknown setting {k}")
        setattr(s, k, v)
    return s


def version() -> str:
    return lib().acs_version().decode()


class Problem:
    """Host copy of (A, b, c, K) inside the library (acs_problem)."""

    def __init__(self, m, n, row_ptr, col_idx, val, b, c, n_orth, soc_sizes=()):
        self._keep = (
            np.ascontiguousarray(row_ptr, dtype=np.int64), np.ascontiguousarray(col_idx, dtype=np.int32),
            np.ascontiguousarray(val, dtype=np.float64), np.ascontiguousarray(b, dtype=np.float64),
            np.ascontiguousarray(c, dtype=np.float64), np.ascontiguousarray(soc_sizes, dtype=np.int32),
        )
        rp, ci, v, bb, cc, ss = self._keep
        self.m, self.n = int(m), int(n)
        self.n_orth = int(n_orth)
        self.soc_sizes = ss
        if len(ci) != len(v):
            raise AcsError(ACS_ERR_ARG, "col_idx and val differ in length")
        if len(rp) != self.m + 1:
            raise AcsError(ACS_ERR_ARG, "row_ptr must have m+1 entries")
        h = P()
        _check(lib().acs_problem_create(self.m, self.n, len(ci), rp.ctypes.data_as(I64P),
                                        ci.ctypes.data_as(I32P), v.ctypes.data_as(DP), bb.ctypes.data_as(DP),
                                        cc.ctypes.data_as(DP), self.n_orth, len(ss), ss.ctypes.data_as(I32P),
                                        ctypes.byref(h)))
        self.handle = h
        self._keep = None  # the library copied everything

    @classmethod
    def from_synth(cls, p) -> "Problem":
        if hasattr(p, "A"):
            return cls.from_dense(p.A, p.b, p.c, p.n_orth, p.soc_sizes)
        return cls(p.m, p.n, p.row_ptr, p.col_idx, p.val, p.b, p.c, p.n_orth, p.soc_sizes)

    @classmethod
    def from_dense(cls, A, b, c, n_orth, soc_sizes=()) -> "Problem":
        """Dense A (m x n, row-major) through acs_problem_create_dense."""
        self = cls.__new__(cls)
        a = np.ascontiguousarray(A, dtype=np.float64)
        if a.ndim != 2:
            raise AcsError(ACS_ERR_ARG, "A must be a 2-D array")
        bb = np.ascontiguousarray(b, dtype=np.float64)
        cc = np.ascontiguousarray(c, dtype=np.float64)
        ss = np.ascontiguousarray(soc_sizes, dtype=np.int32)
        self.m, self.n = int(a.shape[0]), int(a.shape[1])
        if len(bb) != self.m or len(cc) != self.n:
            raise AcsError(ACS_ERR_ARG, "b must have m entries and c n entries")
        self.n_orth = int(n_orth)
        self.soc_sizes = ss
        h = P()
        _check(lib().acs_problem_create_dense(self.m, self.n, a.ctypes.data_as(DP), bb.ctypes.data_as(DP),
                                              cc.ctypes.data_as(DP), self.n_orth, len(ss),
                                              ss.ctypes.data_as(I32P), ctypes.byref(h)))
        self.handle = h
        self._keep = None
        return self

    def device_bytes(self, precision: int = PREC_MIXED) -> int:
        return int(lib().acs_problem_device_bytes(self.handle, precision))

    def factor_bytes(self) -> int:
        return int(lib().acs_problem_factor_bytes(self.handle))

    def batch_device_bytes(self) -> int:
        return int(lib().acs_batch_device_bytes(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            lib().acs_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class State:
    """Resident solver state on the GPU (acs_state)."""

    def __init__(self, problem: Problem, settings: Optional[Settings] = None, stream: int = 0, **kw):
        if settings is None:
            settings = default_settings(**kw)
        self.problem = problem
        self.settings = settings
        h = P()
        _check(lib().acs_state_create(problem.handle, ctypes.byref(settings), P(stream or None), ctypes.byref(h)))
        self.handle = h

    def set(self, l: int, s_prev, s, O, w):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (s_prev, s, O, w)]
        _check(lib().acs_state_set(self.handle, int(l), *[_dptr(a) for a in arrs]))

    def step(self, iters: int):
        _check(lib().acs_state_step(self.handle, int(iters)))

    def solve(self) -> Info:
        info = Info()
        _check(lib().acs_state_solve(self.handle, ctypes.byref(info)))
        return info

    def info(self) -> Info:
        info = Info()
        _check(lib().acs_state_info(self.handle, ctypes.byref(info)))
        return info

    def get(self, xyz: bool = True) -> dict:
        m, n = self.problem.m, self.problem.n
        out = {k: np.empty(n) for k in ("s_prev", "s", "O")}
        out["w"] = np.empty(m)
        if xyz:
            out["x"], out["z"], out["y"] = np.empty(n), np.empty(n), np.empty(m)
        l = ctypes.c_int32()
        _check(lib().acs_state_get(self.handle, ctypes.byref(l), _dptr(out["s_prev"]), _dptr(out["s"]),
                                   _dptr(out["O"]), _dptr(out["w"]), _dptr(out.get("x")), _dptr(out.get("y")),
                                   _dptr(out.get("z"))))
        out["l"] = int(l.value)
        return out

    def spmv(self, which: int, x_ptr: int, y_ptr: int, reps: int = 1) -> float:
        ms = ctypes.c_double()
        _check(lib().acs_state_spmv(self.handle, int(which), P(x_ptr), P(y_ptr), int(reps), ctypes.byref(ms)))
        return ms.value

    def profile(self, classes=True):
        """Time kernel classes with HIP events: True = every class, False = stop,
        or an iterable of KC_* classes."""
        if classes is True:
            mask = PROF_ALL
        elif classes is False or classes is None:
            mask = 0
        else:
            mask = 0
            for k in classes:
                mask |= 1 << int(k)
        _check(lib().acs_state_profile(self.handle, mask))

    def normal_inverse(self) -> np.ndarray:
        """(A O^2 A^T)^+ of the last factorization (direct projection only)."""
        m = self.problem.m
        out = np.empty((m, m))
        _check(lib().acs_state_normal_inverse(self.handle, _dptr(out)))
        return out

    def timing(self, cls: int) -> Tuple[int, float]:
        cnt = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(lib().acs_state_timing(self.handle, int(cls), ctypes.byref(cnt), ctypes.byref(ms)))
        return int(cnt.value), float(ms.value)

    def close(self):
        if getattr(self, "handle", None):
            lib().acs_state_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(problem: Problem, settings: Optional[Settings] = None, stream: int = 0, **kw):
    """One-shot solve; returns (x, y, z, info)."""
    if settings is None:
        settings = default_settings(**kw)
    x, z, y = np.empty(problem.n), np.empty(problem.n), np.empty(problem.m)
    info = Info()
    _check(lib().acs_solve(problem.handle, ctypes.byref(settings), _dptr(x), _dptr(y), _dptr(z), ctypes.byref(info),
                           P(stream or None)))
    return x, y, z, info


def solve_device(problem: Problem, x_ptr: int, y_ptr: int, z_ptr: int, stream: int = 0,
                 settings: Optional[Settings] = None, **kw) -> Info:
    """One-shot solve into caller-owned device buffers (addresses of float64
    device arrays: x, z of length n, y of length m; 0 = not wanted) on
    `stream` (a hipStream_t address, 0 = the library's own)."""
    if settings is None:
        settings = default_settings(**kw)
    info = Info()
    _check(lib().acs_solve_device(problem.handle, ctypes.byref(settings), P(x_ptr or None), P(y_ptr or None),
                                  P(z_ptr or None), ctypes.byref(info), P(stream or None)))
    return info


def solve_device_noalloc(problem: Problem, x_ptr: int, y_ptr: int, z_ptr: int, stream: int = 0,
                         settings: Optional[Settings] = None, **kw) -> Info:
    """solve_device without device allocations (acs_solve_device_noalloc:
    the instance lives in the library's fixed 64 MiB scratch array)."""
    if settings is None:
        settings = default_settings(**kw)
    info = Info()
    _check(lib().acs_solve_device_noalloc(problem.handle, ctypes.byref(settings), P(x_ptr or None),
                                          P(y_ptr or None), P(z_ptr or None), ctypes.byref(info),
                                          P(stream or None)))
    return info


class Batch:
    """Many independent problems solved by one persistent kernel (acs_batch)."""

    def __init__(self, problems, settings: Optional[Settings] = None, stream: int = 0, **kw):
        if settings is None:
            settings = default_settings(**kw)
        self.problems = list(problems)
        self.settings = settings
        arr = (P * len(self.problems))(*[p.handle for p in self.problems])
        h = P()
        _check(lib().acs_batch_create(len(self.problems), arr, ctypes.byref(settings), P(stream or None),
                                      ctypes.byref(h)))
        self.handle = h

    def autotune(self, sample: int = 8, iters: int = 20, cache_path: Optional[str] = None):
        _check(lib().acs_batch_autotune(self.handle, int(sample), int(iters),
                                        cache_path.encode() if cache_path else None))

    def run(self, budget: int, use_graph: bool = True) -> float:
        ms = ctypes.c_double()
        _check(lib().acs_batch_run(self.handle, int(budget), 1 if use_graph else 0, ctypes.byref(ms)))
        return ms.value

    def result(self, i: int, xyz: bool = True):
        p = self.problems[i]
        info = Info()
        x = np.empty(p.n) if xyz else None
        z = np.empty(p.n) if xyz else None
        y = np.empty(p.m) if xyz else None
        _check(lib().acs_batch_result(self.handle, int(i), _dptr(x), _dptr(y), _dptr(z), ctypes.byref(info)))
        return x, y, z, info

    def state(self, i: int) -> dict:
        p = self.problems[i]
        out = {k: np.empty(p.n) for k in ("s_prev", "s", "O")}
        out["w"], out["dsq"] = np.empty(p.m), np.empty(p.m)
        l = ctypes.c_int32()
        _check(lib().acs_batch_state_get(self.handle, int(i), ctypes.byref(l), _dptr(out["s_prev"]), _dptr(out["s"]),
                                         _dptr(out["O"]), _dptr(out["w"]), _dptr(out["dsq"])))
        out["l"] = int(l.value)
        return out

    def lanes(self, i: int):
        a, t = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().acs_batch_lanes(self.handle, int(i), ctypes.byref(a), ctypes.byref(t)))
        return a.value, t.value

    def close(self):
        if getattr(self, "handle", None):
            lib().acs_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop (acs_server)."""

    def __init__(self, hbm_budget: int = 64 << 30, max_slots: int = 256, small_nnz: int = 20_000, workers: int = 6,
                 tick_iters: int = 50):
        h = P()
        _check(lib().acs_server_create(int(hbm_budget), int(max_slots), int(small_nnz), int(workers),
                                       int(tick_iters), ctypes.byref(h)))
        self.handle = h
        self._shapes = {}

    def submit(self, problem: Problem, settings: Optional[Settings] = None, **kw) -> int:
        if settings is None:
            settings = default_settings(**kw)
        t = ctypes.c_uint64()
        _check(lib().acs_server_submit(self.handle, problem.handle, ctypes.byref(settings), ctypes.byref(t)))
        self._shapes[t.value] = (problem.m, problem.n)
        return t.value

    def _fetch(self, fn, ticket, *extra):
        m, n = self._shapes[ticket]
        x, z, y = np.empty(n), np.empty(n), np.empty(m)
        info = Info()
        rc = _check(fn(self.handle, ctypes.c_uint64(ticket), *extra, _dptr(x), _dptr(y), _dptr(z), ctypes.byref(info)))
        if rc == ACS_PENDING:
            return None
        del self._shapes[ticket]
        return x, y, z, info

    def poll(self, ticket: int):
        return self._fetch(lib().acs_server_poll, ticket)

    def wait(self, ticket: int, timeout_ms: int = -1):
        return self._fetch(lib().acs_server_wait, ticket, ctypes.c_int32(timeout_ms))

    def cancel(self, ticket: int):
        _check(lib().acs_server_cancel(self.handle, ctypes.c_uint64(ticket)))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().acs_server_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_ if k != "reserved"}

    def close(self):
        if getattr(self, "handle", None):
            lib().acs_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
