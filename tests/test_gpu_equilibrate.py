"""GPU parity of the Sinkhorn-Knopp equilibration (settings.equilibrate, Sec.
III: A_hat = D A E) against the FP64 oracle, through the C ABI.

* the factors: E after the sweeps, element by element against the oracle's
  sinkhorn_knopp_l2 (both FP64; only summation order differs);
* 20 iterations from the initial state (the l = 1 conditioning included)
  against Algorithm 2 run literally on (D A E, D b, E c);
* a conditioning event of the preconditioned run (the ratio of x_hat, z_hat);
* full solves: KKT of the returned (x, y, z) on the original problem
  recomputed by the oracle, objective against the planted optimum;
* the server's worker path bitwise equal to acs_solve; the batch kernel and
  dense problems refuse the setting.
"""
import numpy as np
import pytest

from oracle.alg2 import default_parameters
from oracle.cones import abs_K
from oracle.equilibrate import EquilibratedAlgorithm2, sinkhorn_knopp_l2
from oracle.kkt import kkt_errors
from paper_2103_00736_amd import acs, synth
from tests._parity import assert_close, assert_iterate, errors, fmt, obj_err

pytestmark = pytest.mark.gpu

SWEEPS = 25


def _edge():
    """Empty rows and columns, and cones of several sizes."""
    p = synth.socp_percol(60, 200, 2, 77, 3, 9, 0.6)
    return p


PROBLEMS = {
    "lp_powerlaw": lambda: synth.config1(scale=0.002),
    "socp": lambda: synth.config2(scale=0.002),
    "sparse_empty": lambda: synth.lp_uniform(50, 125, 62, 8, name="sparse_empty"),
    "socp_small": _edge,
}


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert acs.lib().acs_init(0) == acs.ACS_OK, acs.lib().acs_last_error()


def _oracle(p, sweeps=SWEEPS):
    A = p.scipy_csr()
    d, e = sinkhorn_knopp_l2(A, p.n_orth, p.soc_sizes, sweeps)
    t, L = default_parameters(p.soc_sizes)
    return EquilibratedAlgorithm2(A, p.b, p.c, p.n_orth, p.soc_sizes, d, e, t=t, schedule=L), d, e


def _scaled_errors(p, g, ref_alg, O):
    """Errors in the variables of the iteration (Sec. IV's scaled problem): s;
    the pair (x/O, O z) = ((p + s+)/2, (p - s+)/(2 mu)) as one vector, since
    it is a fixed linear map of (p, s+) and each half on its own can be small
    against the other; and O A^T y, measured against the scaled cost O c that
    it balances.  Returns those errors and, for the record only, the errors of
    x, z and A^T y themselves: the equilibration's E has no cap (on the
    row-scaled LP it spans 1e9), and x_j, z_j, (A^T y)_j carry O_j or 1/O_j
    times the scaled iterate's error."""
    A = p.scipy_csr()
    gy, ry = A.T @ g["y"], A.T @ ref_alg.dual_multiplier()
    gxz = np.concatenate([g["x"] / O, O * g["z"]])
    rxz = np.concatenate([ref_alg.x / O, O * ref_alg.z])
    errs = errors({"s": g["s"], "(x/O, O z)": gxz}, {"s": ref_alg.s, "(x/O, O z)": rxz}, ("s", "(x/O, O z)"))
    d, oc = O * (gy - ry), O * p.c
    errs["O A^T y"] = (float(np.linalg.norm(d) / np.linalg.norm(oc)), float(np.abs(d).max() / np.abs(oc).max()))
    raw = errors({"x": g["x"], "z": g["z"], "A^T y": gy}, {"x": ref_alg.x, "z": ref_alg.z, "A^T y": ry},
                 ("x", "z", "A^T y"))
    return errs, raw


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_factors_match_oracle(name):
    p = PROBLEMS[name]()
    st = acs.State(acs.Problem.from_synth(p), precision=acs.PREC_FP64, equilibrate=1, eq_sweeps=SWEEPS)
    g = st.get(xyz=False)
    _, _, e = _oracle(p)
    err = float(np.max(np.abs(g["O"] - e) / e))
    print(f"{name}: E relative error {err:.2e}, E range {e.min():.3e} .. {e.max():.3e}")
    assert g["l"] == 0
    assert err <= 1e-12
    # the initial state is x = E e_K, z = E^{-1} e_K: one plain step conditions to O = E
    st0 = acs.State(acs.Problem.from_synth(p), precision=acs.PREC_FP64, equilibrate=1, eq_sweeps=0)
    assert np.array_equal(st0.get(xyz=False)["O"], np.ones(p.n))


# sparse_empty has rows and columns without total support: no balanced scaling
# exists, the sweeps drift and E spans 1e11, beyond what FP32 values of A_s
# resolve; it is compared in FP64 only
@pytest.mark.parametrize("name,prec", [(n, acs.PREC_FP64) for n in ("lp_powerlaw", "socp", "sparse_empty")] +
                         [(n, acs.PREC_MIXED) for n in ("lp_powerlaw", "socp")])
def test_k_iterations_match_oracle(name, prec):
    """20 iterations from the initial state, tight CG: s and O against the
    literal run on the preconditioned problem; x/O, z and A^T y of the last."""
    p = PROBLEMS[name]()
    k = 20
    alg, d, e = _oracle(p)
    for _ in range(k):
        alg.step()
    st = acs.State(acs.Problem.from_synth(p), precision=prec, equilibrate=1, eq_sweeps=SWEEPS, cg_max=4000,
                   cg_reduce=1e-13 if prec == acs.PREC_FP64 else 1e-7, check_every=1000000)
    st.step(k)
    g = st.get()
    errs, raw = _scaled_errors(p, g, alg, alg.O)
    oerr = errors(g, {"O": alg.O}, ("O",))
    print(f"{name} prec={prec}: {fmt(oerr)} {fmt(errs)}; original variables {fmt(raw)}")
    assert g["l"] == k
    assert_close(oerr, 1e-9, name)
    # twenty steps compound the one-step error: the bars of one step, times ten in FP64
    if prec == acs.PREC_FP64:
        assert_close(errs, 1e-8, name, elem_tol=1e-7)
    else:
        assert_close(errs, 1e-5, name)


@pytest.mark.parametrize("name", ["lp_powerlaw", "socp"])
def test_conditioning_event_parity(name):
    """The event at the second member of L on the preconditioned run: O = E O_hat
    with O_hat from the ratio of x_hat, z_hat."""
    p = PROBLEMS[name]()
    t, L = default_parameters(p.soc_sizes)
    l_event = L.first + L.every
    alg, d, e = _oracle(p)
    s_prev = None
    while alg.l < l_event - 1:
        s_prev = alg.s.copy()
        alg.step()
    s, O = alg.s.copy(), alg.O.copy()
    w = -alg.dual_multiplier()
    # the oracle from exactly the shared state: x_hat, z_hat of the last iteration
    pp = abs_K(s_prev, p.n_orth, p.soc_sizes)
    O_hat = alg.inner.O.copy()
    alg.inner.x = O_hat * (pp + s) / 2.0
    alg.inner.z = (pp - s) / (2.0 * O_hat)
    alg.step()
    st = acs.State(acs.Problem.from_synth(p), precision=acs.PREC_FP64, equilibrate=1, eq_sweeps=SWEEPS,
                   cg_max=2000, cg_reduce=1e-13)
    st.set(l_event - 1, s_prev, s, O, w)
    st.step(1)
    g = st.get()
    oerr = errors(g, {"O": alg.O}, ("O",))
    errs, raw = _scaled_errors(p, g, alg, alg.O)
    print(f"{name}: {fmt(oerr)} {fmt(errs)}; original variables {fmt(raw)}; "
          f"O_hat range {np.log(alg.inner.O.max() / alg.inner.O.min()):.3f}")
    assert_close(oerr, 1e-9, name)
    assert_iterate(errs, True, name)


# The row-scaled power-law LP (row scales 10^+-3) gets column scales E that
# span about 1e9: the FP32 CG of the mixed path then sits at the edge of what
# its refinement can recover, and whether the solve converges within 20000
# iterations turns on the last bits of ||t||^2 (10740 iterations on 8 column
# slices with one summation order, a stall near KKT 1e-1 with another).  That
# case runs the FP64 path (about 3800 iterations with either order); the SOCP
# the mixed one.
@pytest.mark.parametrize("name,precision", [("lp_powerlaw", acs.PREC_FP64), ("socp", acs.PREC_MIXED)])
def test_equilibrated_solve(name, precision):
    p = PROBLEMS[name]()
    prob = acs.Problem.from_synth(p)
    x, y, z, info = acs.solve(prob, equilibrate=1, eps_kkt=1e-4, max_iter=20000, precision=precision)
    rec = kkt_errors(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, x, y, z)
    oe = obj_err(rec["pobj"], p.p_star)
    _, _, _, plain = acs.solve(prob, eps_kkt=1e-4, max_iter=20000, precision=precision)
    print(f"{name}: equilibrated {info.iterations} it ({info.cg_steps} CG) oracle kkt {rec['kkt']:.2e} "
          f"obj_err {oe:.1e}; plain {plain.iterations} it ({plain.cg_steps} CG)")
    assert info.status == acs.SOLVED
    assert rec["kkt"] <= 1.05e-4
    assert oe <= 1e-4


def test_server_worker_path_and_refusals():
    # 10% density: every row and column has nonzeros, so the balance exists
    p = synth.lp_uniform(100, 250, 2500, 21, name="lp_dense10")
    prob = acs.Problem.from_synth(p)
    srv = acs.Server(hbm_budget=1 << 30, max_slots=8, small_nnz=1 << 30, workers=2, tick_iters=25)
    ticket = srv.submit(prob, equilibrate=1, eps_kkt=1e-4)
    x, y, z, info = srv.wait(ticket, 120_000)
    srv.close()
    xa, ya, za, ia = acs.solve(prob, equilibrate=1, eps_kkt=1e-4)
    assert info.status == ia.status == acs.SOLVED and info.iterations == ia.iterations
    assert np.array_equal(x, xa) and np.array_equal(y, ya) and np.array_equal(z, za)
    with pytest.raises(acs.AcsError) as e:
        acs.Batch([prob], equilibrate=1)
    assert e.value.code == acs.ACS_ERR_ARG
    dense = acs.Problem.from_synth(synth.e3_lp(200))
    with pytest.raises(acs.AcsError) as e:
        acs.solve(dense, equilibrate=1)
    assert e.value.code == acs.ACS_ERR_ARG
