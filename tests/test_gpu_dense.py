"""GPU checks of the dense path (the paper's random LP and SOCP instances,
Sec. V-B and V-D) through the C ABI: one-iteration and conditioning-event
parity against the oracle, full solves against the oracle's KKT and SciPy's
LP optimum, the dense products on sampled rows at a large size, the same
matrix as dense and as CSR, and dense requests in the server."""
import numpy as np
import pytest
from scipy.optimize import linprog

from oracle.alg2 import Algorithm2, default_parameters, one_iteration
from oracle.cones import abs_K
from oracle.kkt import kkt_errors
from paper_2103_00736_amd import acs, synth
from tests._parity import assert_close, assert_iterate, errors, fmt, iterate_errors, obj_err as _obj_err

pytestmark = pytest.mark.gpu


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert acs.lib().acs_init(0) == acs.ACS_OK, acs.lib().acs_last_error()


PROBLEMS = {
    "e3_lp": lambda: synth.e3_lp(400),
    "e6_socp_h4": lambda: synth.e6_socp(400, 4),
    "e6_socp_h10": lambda: synth.e6_socp(403, 10),  # with an orthant remainder
}


def _oracle_state(p, iters):
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
def test_dense_one_iteration_parity(name, prec, after_event):
    p = PROBLEMS[name]()
    t, L = default_parameters(p.soc_sizes)
    l0 = L.first + 17 if after_event else 57
    alg, s_prev, s, O, w = _oracle_state(p, l0)
    if prec == acs.PREC_MIXED:
        s_prev, s = _f32(s_prev), _f32(s)
    st = acs.State(acs.Problem.from_synth(p), precision=prec, cg_max=3000,
                   cg_reduce=1e-13 if prec == acs.PREC_FP64 else 1e-7)
    st.set(l0, s_prev, s, O, w)
    st.step(1)
    g = st.get()
    ref = one_iteration(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, 1.0, s, O)
    errs = iterate_errors(g, ref, O)
    print(name, prec, l0, "(normwise/elementwise)", fmt(errs))
    assert_iterate(errs, prec == acs.PREC_FP64, name)


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_dense_conditioning_event_parity(name):
    p = PROBLEMS[name]()
    t, L = default_parameters(p.soc_sizes)
    l_event = L.first + L.every
    alg, s_prev, s, O, w = _oracle_state(p, l_event - 1)
    pp = abs_K(s_prev, p.n_orth, p.soc_sizes)
    alg.x = O * (pp + s) / 2.0
    alg.z = (pp - s) / (2.0 * O)
    alg.l = l_event - 1
    alg.step()
    st = acs.State(acs.Problem.from_synth(p), precision=acs.PREC_FP64, cg_max=3000, cg_reduce=1e-13)
    st.set(l_event - 1, s_prev, s, O, w)
    st.step(1)
    g = st.get()
    errs = errors(g, {"O": alg.O, "s": alg.s}, ("O", "s"))
    print(name, fmt(errs))
    assert_close(errs, 1e-9, name)


def _check_solve(p, x, y, z, info, eps):
    rec = kkt_errors(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, x, y, z)
    print(f"{p.name}: status={info.status} it={info.iterations} cg={info.cg_steps} gpu_kkt={info.kkt:.2e} "
          f"oracle_kkt={rec['kkt']:.2e} pobj={rec['pobj']:.8f} solve_ms={info.solve_ms:.1f}")
    assert info.status == acs.SOLVED
    assert rec["kkt"] <= eps
    assert abs(info.kkt - rec["kkt"]) <= 1e-6 + 0.02 * rec["kkt"]
    return rec


def test_dense_lp_fp64_matches_highs():
    p = synth.e3_lp(300)
    x, y, z, info = acs.solve(acs.Problem.from_synth(p), precision=acs.PREC_FP64, eps_kkt=1e-7, max_iter=20000)
    rec = _check_solve(p, x, y, z, info, 1.05e-7)
    lp = linprog(p.c, A_eq=p.A, b_eq=p.b, bounds=(0, None), method="highs")
    assert abs(rec["pobj"] - lp.fun) <= 1e-5 * (1 + abs(lp.fun))


@pytest.mark.parametrize("make", [lambda: synth.e3_lp(1500), lambda: synth.e6_socp(1500, 10),
                                  lambda: synth.e6_socp(1000, 4)])
def test_dense_mixed_solves(make):
    p = make()
    x, y, z, info = acs.solve(acs.Problem.from_synth(p), eps_kkt=1e-4, max_iter=20000)
    rec = _check_solve(p, x, y, z, info, 1.05e-4)
    if not p.is_socp:
        lp = linprog(p.c, A_eq=p.A, b_eq=p.b, bounds=(0, None), method="highs")
        assert _obj_err(rec["pobj"], lp.fun) <= 1e-4
    else:  # against the oracle's own solution of the same SOCP
        t, L = default_parameters(p.soc_sizes)
        alg = Algorithm2(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, mu=1.0, t=t, schedule=L)
        alg.run(20000, eps=1e-7, check_every=10)
        assert _obj_err(rec["pobj"], p.c @ alg.x) <= 1e-4


def test_dense_and_csr_give_the_same_iteration():
    p = synth.e3_lp(500)
    import scipy.sparse as sp
    A = sp.csr_matrix(p.A)
    sparse = acs.Problem(p.m, p.n, A.indptr, A.indices, A.data, p.b, p.c, p.n_orth)
    dense = acs.Problem.from_synth(p)
    outs = []
    for h in (sparse, dense):
        st = acs.State(h, precision=acs.PREC_FP64, cg_max=3000, cg_reduce=1e-13)
        st.step(320)  # through the first conditioning event
        outs.append(st.get())
    for k in ("s", "x", "z", "y", "O"):
        assert _rel(outs[1][k], outs[0][k]) <= 1e-8, k


def test_dense_products_on_sampled_rows_large():
    import torch

    p = synth.e3_lp(8000)  # 6400 x 8000, 51M entries
    st = acs.State(acs.Problem.from_synth(p))
    st.step(301)  # past the first conditioning: O spans e^9.2
    g = st.get(xyz=False)
    O = g["O"]
    d = 1.0 / np.sqrt((p.A * p.A) @ (O * O))
    rng = np.random.default_rng(2)
    dev = torch.device("cuda:0")
    xn = rng.standard_normal(p.n).astype(np.float32)
    xm = rng.standard_normal(p.m).astype(np.float32)
    ym = torch.empty(p.m, dtype=torch.float32, device=dev)
    yn = torch.empty(p.n, dtype=torch.float32, device=dev)
    st.spmv(0, torch.from_numpy(xn).to(dev).data_ptr(), ym.data_ptr())
    st.spmv(1, torch.from_numpy(xm).to(dev).data_ptr(), yn.data_ptr())
    torch.cuda.synchronize()
    ym, yn = ym.cpu().numpy(), yn.cpu().numpy()
    for i in rng.choice(p.m, 300, replace=False):
        terms = d[i] * p.A[i] * O * xn
        assert abs(ym[i] - terms.sum()) <= 1e-5 * np.abs(terms).sum(), i
    for j in rng.choice(p.n, 300, replace=False):
        terms = d * p.A[:, j] * O[j] * xm
        assert abs(yn[j] - terms.sum()) <= 1e-5 * np.abs(terms).sum(), j


def test_dense_request_in_server_and_batch_rejects():
    p = synth.e3_lp(600)
    h = acs.Problem.from_synth(p)
    srv = acs.Server(hbm_budget=1 << 30, max_slots=4, small_nnz=1 << 30, workers=1, tick_iters=25)
    ticket = srv.submit(h, eps_kkt=1e-4)
    x, y, z, info = srv.wait(ticket, 120_000)
    xa, ya, za, ia = acs.solve(h, eps_kkt=1e-4)
    assert info.status == acs.SOLVED and np.array_equal(x, xa) and np.array_equal(y, ya)
    srv.close()
    with pytest.raises(acs.AcsError) as ei:
        acs.Batch([h])
    assert ei.value.code == acs.ACS_ERR_ARG
