"""GPU checks of the direct projection (M = A_s A_s^T formed and inverted in
FP64 at every conditioning event, w += M^{-1} r each iteration) through the
C ABI: the inverse against the oracle's (B B^T)^+, one iteration and a
conditioning event against the oracle's exact-projection iteration, whole
trajectories through several events, full solves, tile-boundary sizes,
dependent rows, and a property check at the dense LP's full size."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.alg2 import Algorithm2, Schedule, conditioning_ratio, default_parameters, one_iteration
from oracle.cones import abs_K
from oracle.kkt import kkt_errors
from oracle.subspace import RangeProjector
from paper_2103_00736_amd import acs, synth
from tests._parity import assert_close, errors, fmt, obj_err as _obj_err

pytestmark = pytest.mark.gpu

FACTOR = dict(projection=acs.PROJ_FACTOR)


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert acs.lib().acs_init(0) == acs.ACS_OK, acs.lib().acs_last_error()


class _Sparse:
    """A planted sparse LP from a dense FP32 array (rows may be empty or repeated)."""

    def __init__(self, A, seed, name):
        rng = np.random.default_rng(seed)
        self.A = _f32(A)
        self.m, self.n = A.shape
        x0 = np.where(rng.random(self.n) < 0.5, rng.random(self.n) + 0.1, 0.0)
        z0 = np.where(x0 > 0, 0.0, rng.random(self.n) + 0.1)
        y0 = rng.standard_normal(self.m)
        self.b = self.A @ x0
        self.c = self.A.T @ y0 + z0
        self.n_orth, self.soc_sizes, self.name = self.n, np.zeros(0, np.int32), name

    def scipy_csr(self):
        return sp.csr_matrix(self.A)

    def handle(self):
        C = self.scipy_csr()
        return acs.Problem(self.m, self.n, C.indptr, C.indices, C.data, self.b, self.c, self.n_orth)


def _sparse_edge():
    """200 x 500 at 2% density with 3 empty rows and one row repeated."""
    rng = np.random.default_rng(3)
    A = np.where(rng.random((200, 500)) < 0.02, rng.standard_normal((200, 500)), 0.0)
    A[[5, 77, 150]] = 0.0
    A[120] = A[40]
    return _Sparse(A, 4, "sparse_edge")


def _handle(p):
    return p.handle() if isinstance(p, _Sparse) else acs.Problem.from_synth(p)


PROBLEMS = {
    "e3_lp_560x700": lambda: synth.e3_lp(700),         # 9 pivot blocks, the last one ragged
    "e6_socp_h10": lambda: synth.e6_socp(403, 10),     # dense SOCP with an orthant remainder
    "sparse_lp": lambda: synth.lp_uniform(200, 500, 2000, 9),
    "sparse_edge": _sparse_edge,
}


def _random_state(p, seed):
    """(s_prev, s, O, w) with O constant on every cone, spread like a conditioned scaling."""
    rng = np.random.default_rng(seed)
    n, m = p.n, p.m
    units = p.n_orth + len(p.soc_sizes)
    ou = np.exp(rng.uniform(-3.0, 3.0, units))
    O = np.repeat(ou, np.r_[np.ones(p.n_orth, dtype=int), np.asarray(p.soc_sizes, dtype=int)])
    return rng.standard_normal(n), rng.standard_normal(n), O, rng.standard_normal(m)


# problems whose A has dependent rows: there (B B^T)^+ is not the only
# generalized inverse, and only the projector B^T X B (and A^T y) is unique
DEPENDENT = {"sparse_edge"}


def _kappa(p, O):
    """Condition number of the unit-diagonal normal matrix D^-1/2 A O^2 A^T D^-1/2
    on its range (empty rows and null directions left out)."""
    B = RangeProjector(p.scipy_csr(), O, method="exact").B.toarray()
    G = B @ B.T
    live = np.abs(B).sum(axis=1) > 0
    dg = 1.0 / np.sqrt(np.diag(G)[live])
    ev = np.linalg.eigvalsh(G[np.ix_(live, live)] * dg[:, None] * dg[None, :])
    ev = ev[ev > ev.max() * 1e-12]
    return float(ev.max() / ev.min())


def _fp64_bar(p, O, name=""):
    """Relative error bar of an FP64 iteration whose projection solves with the
    normal matrix: ten times kappa times the unit roundoff 2^-53; with
    dependent rows the roundoff left in the null direction (about m u) is
    divided by the smallest nonzero eigenvalue, one more factor m."""
    bar = 10.0 * _kappa(p, O) * 2.0 ** -53
    if name in DEPENDENT:
        bar *= p.m
    return max(1e-13, bar)


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("prec", [acs.PREC_FP64, acs.PREC_MIXED])
def test_normal_inverse_matches_oracle(name, prec):
    p = PROBLEMS[name]()
    s_prev, s, O, w = _random_state(p, 1)
    st = acs.State(_handle(p), precision=prec, **FACTOR)
    st.set(57, s_prev, s, O, w)
    X = st.normal_inverse()
    proj = RangeProjector(p.scipy_csr(), O, method="exact")
    Xo = proj.normal_pinv()
    B = proj.B.toarray()
    G = B @ B.T
    live = np.abs(B).sum(axis=1) > 0
    w_, V = np.linalg.eigh(G[np.ix_(live, live)])
    pos = w_[w_ > w_.max() * 1e-12]
    cond = pos.max() / pos.min()
    Pj, Pjo = B.T @ X @ B, B.T @ Xo @ B
    perr = np.abs(Pj - Pjo).max() / np.abs(Pjo).max()
    gig = np.abs(G @ X @ G - G).max() / np.abs(G).max()
    print(f"{name} prec={prec} m={p.m} cond={cond:.2e} |P-Po|={perr:.2e} |GXG-G|={gig:.2e}")
    assert np.all(X[~live] == 0) and np.all(X[:, ~live] == 0)
    assert np.array_equal(X, X.T)
    bound = 1e-14 * cond * p.m
    assert perr <= bound and gig <= bound
    if name not in DEPENDENT:
        err = np.abs(X - Xo).max() / np.abs(Xo).max()
        eye = np.abs((G @ X)[np.ix_(live, live)] - np.eye(live.sum())).max()
        print(f"   |X-Xo|/|Xo|={err:.2e} |GX-I|={eye:.2e}")
        assert err <= bound and eye <= bound


def _oracle_at(p, iters):
    t, L = default_parameters(p.soc_sizes)
    alg = Algorithm2(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, mu=1.0, t=t, schedule=L)
    s_prev = None
    for _ in range(iters):
        s_prev = alg.s.copy()
        alg.step()
    return alg, s_prev, alg.s.copy(), alg.O.copy(), -alg.dual_multiplier()


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("prec", [acs.PREC_FP64, acs.PREC_MIXED])
@pytest.mark.parametrize("after_event", [False, True])
def test_factor_one_iteration_parity(name, prec, after_event):
    p = PROBLEMS[name]()
    t, L = default_parameters(p.soc_sizes)
    l0 = L.first + 17 if after_event else 57
    alg, s_prev, s, O, w = _oracle_at(p, l0)
    if prec == acs.PREC_MIXED:
        s_prev, s = _f32(s_prev), _f32(s)
    st = acs.State(_handle(p), precision=prec, **FACTOR)
    st.set(l0, s_prev, s, O, w)
    st.step(1)
    g = st.get()
    ref = one_iteration(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, 1.0, s, O)
    errs = errors(g, ref, ("s", "x", "z"))
    A = p.scipy_csr()
    yerrs = errors({"A^T y": A.T @ g["y"]}, {"A^T y": A.T @ ref["y"]}, ("A^T y",))
    if name not in DEPENDENT:
        yerrs.update(errors(g, ref, ("y",)))
    tol = _fp64_bar(p, O, name) if prec == acs.PREC_FP64 else 1e-6
    # y solves the normal equations: its bar carries their conditioning in
    # FP64 (ten times the bar of s); in mixed precision it is the 1e-5 bar
    tol_y = 10 * tol if prec == acs.PREC_FP64 else 1e-5
    print(name, prec, l0, "(normwise/elementwise)", fmt(errs), fmt(yerrs), f"bar {tol:.1e}")
    assert_close(errs, tol, name)
    assert_close(yerrs, tol_y, name)


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_factor_conditioning_event_parity(name):
    """The step that conditions (steps 5-14, then the new factorization) and projects."""
    p = PROBLEMS[name]()
    t, L = default_parameters(p.soc_sizes)
    l_event = L.first + L.every
    alg, s_prev, s, O, w = _oracle_at(p, l_event - 1)
    pp = abs_K(s_prev, p.n_orth, p.soc_sizes)
    alg.x = O * (pp + s) / 2.0
    alg.z = (pp - s) / (2.0 * O)
    alg.l = l_event - 1
    alg.step()
    st = acs.State(_handle(p), precision=acs.PREC_FP64, **FACTOR)
    st.set(l_event - 1, s_prev, s, O, w)
    st.step(1)
    g = st.get()
    bar = _fp64_bar(p, alg.O, name)
    # the new M^{-1} belongs to the new O: compare the projectors
    proj = RangeProjector(p.scipy_csr(), g["O"], method="exact")
    B = proj.B.toarray()
    Pj, Pjo = B.T @ st.normal_inverse() @ B, B.T @ proj.normal_pinv() @ B
    perr = np.abs(Pj - Pjo).max() / np.abs(Pjo).max()
    print(name, f"O {_rel(g['O'], alg.O):.2e} s {_rel(g['s'], alg.s):.2e} bar {bar:.1e} projector {perr:.2e}")
    assert _rel(g["O"], alg.O) <= 1e-10
    assert _rel(g["s"], alg.s) <= bar
    assert perr <= 1e-14 * _kappa(p, g["O"]) * p.m


@pytest.mark.parametrize("name", ["sparse_lp", "e3_lp_560x700", "e6_socp_h10"])
def test_factor_trajectory_through_events(name):
    """80 iterations with events at 1, 30 and 60: the GPU's exact projections keep
    it on the oracle's trajectory.  x and z (the method's output) must agree
    tightly.  The event at 60 sets O from logs of the ratios of steps 5-10,
    whose entries both tend to zero, so it magnifies the tiny difference in x
    and z that the two implementations carry into it: the bar for O and s is
    that difference in log o at l = 59 propagated through step 11 (the log
    range normalisation at most triples it; s = x/O - mu O z follows O)."""
    p = PROBLEMS[name]()
    t, _ = default_parameters(p.soc_sizes)
    L = Schedule(30, 30, 60)
    alg = Algorithm2(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, mu=1.0, t=t, schedule=L)
    st = acs.State(_handle(p), precision=acs.PREC_FP64, check_every=1000000, auto_params=0, t=t, mu=1.0,
                   l_first=30, l_every=30, l_last=60, **FACTOR)
    for _ in range(59):
        alg.step()
    st.step(59)
    g59 = st.get()
    lo_g = np.log(conditioning_ratio(g59["x"], g59["z"], p.n_orth, p.soc_sizes))
    lo_o = np.log(conditioning_ratio(alg.x, alg.z, p.n_orth, p.soc_sizes))
    fin = np.isfinite(lo_g) & np.isfinite(lo_o)
    dlog = float(np.abs(lo_g - lo_o)[fin].max())
    for _ in range(21):
        alg.step()
    st.step(21)
    g = st.get()
    errs = {k: _rel(g[k], getattr(alg, k)) for k in ("s", "O", "x", "z")}
    bar_o = 3.0 * dlog + 1e-12
    bar_s = bar_o * (np.linalg.norm(alg.x / alg.O) + np.linalg.norm(alg.O * alg.z)) / np.linalg.norm(alg.s) + 1e-12
    print(name, {k: f"{v:.2e}" for k, v in errs.items()}, f"dlog(l=59) {dlog:.2e} bar O {bar_o:.1e} s {bar_s:.1e}")
    assert g["l"] == 80
    assert errs["x"] <= 1e-8 and errs["z"] <= 1e-8
    assert errs["O"] <= bar_o and errs["s"] <= bar_s


def _check_solve(p, x, y, z, info, eps):
    rec = kkt_errors(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, x, y, z)
    print(f"{p.name}: status={info.status} it={info.iterations} cg={info.cg_steps} gpu_kkt={info.kkt:.2e} "
          f"oracle_kkt={rec['kkt']:.2e} pobj={rec['pobj']:.8f} solve_ms={info.solve_ms:.1f}")
    assert info.status == acs.SOLVED
    assert rec["kkt"] <= eps
    assert abs(info.kkt - rec["kkt"]) <= 1e-6 + 0.02 * rec["kkt"]
    return rec


@pytest.mark.parametrize("make", [lambda: synth.e3_lp(1500), lambda: synth.e6_socp(1500, 10),
                                  lambda: synth.config0(0)], ids=["e3_lp_1500", "e6_socp_1500", "config0"])
@pytest.mark.parametrize("prec", [acs.PREC_MIXED, acs.PREC_FP64])
def test_factor_full_solve(make, prec):
    p = make()
    eps = 1e-4 if prec == acs.PREC_MIXED else 1e-6
    x, y, z, info = acs.solve(_handle(p), precision=prec, eps_kkt=eps, max_iter=20000, **FACTOR)
    rec = _check_solve(p, x, y, z, info, eps * 1.05)
    assert info.cg_steps == 0
    if hasattr(p, "p_star"):
        assert _obj_err(rec["pobj"], p.p_star) <= 1e-4


@pytest.mark.parametrize("m", [1, 63, 64, 65, 127, 128, 129, 200, 257, 500])
def test_factor_tile_boundaries(m):
    """Orders around the 64-row pivot blocks and the 128-row padding, with
    odd and even block counts (steps are swept in pairs)."""
    n = max(2, int(m * 1.25) + 1)
    rng = np.random.default_rng(m)
    p = _Sparse(rng.uniform(-1, 1, (m, n)), m, f"dense_{m}x{n}")
    s_prev, s, O, w = _random_state(p, m)
    st = acs.State(p.handle(), precision=acs.PREC_FP64, **FACTOR)
    st.set(57, s_prev, s, O, w)
    X = st.normal_inverse()
    Xo = RangeProjector(p.scipy_csr(), O, method="exact").normal_pinv()
    err = np.abs(X - Xo).max() / np.abs(Xo).max()
    kappa = _kappa(p, O)
    st.step(1)
    g = st.get()
    ref = one_iteration(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, 1.0, s, O)
    serr, bar = _rel(g["s"], ref["s"]), _fp64_bar(p, O)
    print(m, f"kappa {kappa:.2e} inverse {err:.2e} s {serr:.2e} bar {bar:.1e}")
    assert err <= 1e-14 * kappa * m + 1e-15
    assert serr <= bar


@pytest.mark.parametrize("n", [700, 2500])
def test_factor_sweep_bitwise_reproducible(n):
    """The sweep's passes run beside the next group's pivots, panels and strips
    on a second stream; the two touch disjoint tiles and W panels, so the
    inverse is the same bit for bit on a refactorization and in a fresh state
    (9 and 32 pivot blocks: one and seven overlapped groups)."""
    p = synth.e3_lp(n)
    s_prev, s, O, w = _random_state(p, 3)
    h = acs.Problem.from_synth(p)
    st = acs.State(h, precision=acs.PREC_FP64, **FACTOR)
    st.set(57, s_prev, s, O, w)
    X1 = st.normal_inverse()
    st.set(57, s_prev, s, O, w)
    X2 = st.normal_inverse()
    st2 = acs.State(h, precision=acs.PREC_FP64, **FACTOR)
    st2.set(57, s_prev, s, O, w)
    X3 = st2.normal_inverse()
    st.close()
    st2.close()
    h.close()
    assert np.isfinite(X1).all()
    assert np.array_equal(X1, X2)
    assert np.array_equal(X1, X3)


def test_factor_dependent_rows_solve():
    """Empty and repeated rows: the skipped pivots leave a pseudo-inverse and
    the solve converges as the oracle's does."""
    p = _sparse_edge()
    x, y, z, info = acs.solve(p.handle(), precision=acs.PREC_FP64, eps_kkt=1e-6, max_iter=20000, **FACTOR)
    _check_solve(p, x, y, z, info, 1.05e-6)


def test_factor_matches_cg_solution():
    """Both projections reach the same objective and dual (unique) on a dense LP."""
    p = synth.e3_lp(1000)
    h = acs.Problem.from_synth(p)
    xf, yf, zf, infof = acs.solve(h, precision=acs.PREC_FP64, eps_kkt=1e-7, max_iter=20000, **FACTOR)
    xc, yc, zc, infoc = acs.solve(h, precision=acs.PREC_FP64, eps_kkt=1e-7, max_iter=20000)
    print(f"iterations factor {infof.iterations} cg {infoc.iterations}; cg steps {infoc.cg_steps}")
    assert infof.status == acs.SOLVED and infoc.status == acs.SOLVED
    assert abs(infof.pobj - infoc.pobj) <= 1e-5 * (1 + abs(infoc.pobj))
    assert _rel(yf, yc) <= 1e-3


def test_factor_state_errors():
    p = synth.lp_uniform(20, 50, 200, 1)
    h = acs.Problem.from_synth(p)
    st = acs.State(h)  # CG state
    with pytest.raises(acs.AcsError) as ei:
        st.normal_inverse()
    assert ei.value.code == acs.ACS_ERR_STATE
    sf = acs.State(h, **FACTOR)  # at l = 0 the first factorization waits for the event at l = 1
    with pytest.raises(acs.AcsError) as ei:
        sf.normal_inverse()
    assert ei.value.code == acs.ACS_ERR_STATE
    sf.step(1)
    assert np.isfinite(sf.normal_inverse()).all()
    with pytest.raises(acs.AcsError) as ei:
        acs.Batch([h], **FACTOR)
    assert ei.value.code == acs.ACS_ERR_ARG
    with pytest.raises(acs.AcsError) as ei:
        acs.State(h, projection=7)
    assert ei.value.code == acs.ACS_ERR_ARG


def test_factor_server_worker_matches_solve():
    p = synth.e3_lp(600)
    h = acs.Problem.from_synth(p)
    x0, y0, z0, i0 = acs.solve(h, eps_kkt=1e-5, max_iter=20000, **FACTOR)
    srv = acs.Server(hbm_budget=8 << 30, max_slots=4, workers=1)
    try:
        t = srv.submit(h, eps_kkt=1e-5, max_iter=20000, **FACTOR)
        x1, y1, z1, i1 = srv.wait(t)
    finally:
        srv.close()
    assert i1.status == acs.SOLVED and i1.iterations == i0.iterations
    assert np.array_equal(x0, x1) and np.array_equal(y0, y1) and np.array_equal(z0, z1)


@pytest.fixture(scope="module")
def full_size_lp():
    return synth.e3_lp(30000)


@pytest.mark.parametrize("prec", [acs.PREC_MIXED, acs.PREC_FP64])
def test_factor_full_size_normal_equations(full_size_lp, prec):
    """At the dense LP's full size (n = 30000, m = 24000; the benchmark runs it
    in mixed precision): the GPU's w solves (A O^2 A^T) w = A O (p - mu O c) - b,
    checked with plain FP64 products.  One step from a random w corrects it by
    M^{-1} r with a residual of about ||I - M M^{-1}|| ||r||; a second step from
    the same s (the warm start of the iteration) refines it.  The bar after the
    second step: FP64, a few hundred units of roundoff; mixed precision, the
    FP32 rounding of v = p - chat - A_s^T w through A O, u32 || |A| O |v| ||."""
    p = full_size_lp
    A = p.A
    s_prev, s, O, w0 = _random_state(p, 7)
    s_prev, s = _f32(s_prev), _f32(s)
    st = acs.State(acs.Problem.from_synth(p), precision=prec, **FACTOR)
    pk = np.abs(s)  # abs_K on the orthant
    rhs = A @ (O * (pk - O * p.c)) - p.b
    nr = np.linalg.norm(rhs)
    res, bars = [], []
    w = w0
    for _ in range(2):
        st.set(57, s_prev, s, O, w)
        st.step(1)
        w_in, w = w, st.get(xyz=False)["w"]
        res.append(np.linalg.norm(A @ (O * O * (A.T @ w)) - rhs) / nr)
        v_in = pk - O * p.c - O * (A.T @ w_in)  # v of this step
        bars.append(2.0 ** -24 * np.linalg.norm(np.abs(A) @ (O * np.abs(v_in))) / nr)
    st.close()
    if prec == acs.PREC_FP64:
        bars = [1e-6, 1e-12]  # one correction from a random w, then one refinement
    print(f"full size prec={prec}: ||M w - rhs|| / ||rhs|| = {res[0]:.2e} (one step), {res[1]:.2e} (two), "
          f"bars {bars[0]:.1e} {bars[1]:.1e}")
    assert res[0] <= bars[0] + 1e-8
    assert res[1] <= bars[1] + 1e-12


def test_projection_auto_picks_by_m():
    """ACS_PROJ_AUTO takes the direct projection for m <= 2048 and the CG
    above: bitwise the explicit choice in each case; the batch kernel takes it
    as CG."""
    small = synth.config0()  # m = 200
    large = synth.config1(scale=0.005)  # m = 2500
    assert small.m <= 2048 < large.m
    for p, explicit in ((small, acs.PROJ_FACTOR), (large, acs.PROJ_CG)):
        h = acs.Problem.from_synth(p)
        a = acs.solve(h, eps_kkt=1e-4, max_iter=20000, projection=acs.PROJ_AUTO)
        b = acs.solve(h, eps_kkt=1e-4, max_iter=20000, projection=explicit)
        assert a[3].status == acs.SOLVED and a[3].iterations == b[3].iterations, p.name
        for u, v in zip(a[:3], b[:3]):
            assert np.array_equal(u, v), p.name
    probs = [synth.config3(i) for i in range(3)]
    hs = [acs.Problem.from_synth(q) for q in probs]
    res = []
    for proj in (acs.PROJ_AUTO, acs.PROJ_CG):
        bt = acs.Batch(hs, eps_kkt=1e-4, max_iter=20000, projection=proj)
        bt.run(20000)
        res.append([bt.result(i) for i in range(len(hs))])
        bt.close()
    for ra, rb in zip(*res):
        assert ra[3].status == acs.SOLVED and ra[3].iterations == rb[3].iterations
        for u, v in zip(ra[:3], rb[:3]):
            assert np.array_equal(u, v)
