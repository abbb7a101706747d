"""GPU parity of the HIP solver against the FP64 oracle, through the C ABI.

* one iteration (steps 16-20) from a shared state, before and after a
  conditioning event, FP64 and mixed precision;
* the conditioning event itself (steps 5-14): O and the re-cast s;
* full solves: KKT of the returned (x, y, z) recomputed by the oracle in FP64,
  objective against the planted optimum (1e-4 relative), z and y against the
  oracle's;
* run-to-run bitwise determinism.

Vectors are compared normwise and element by element (tests/_parity.py).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.alg2 import Algorithm2, Schedule, default_parameters, one_iteration
from oracle.cones import abs_K
from oracle.kkt import kkt_errors
from paper_2103_00736_amd import acs, synth
from tests._parity import assert_close, assert_iterate, errors, fmt, iterate_errors, obj_err as _obj_err

pytestmark = pytest.mark.gpu


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _oracle_run(p, iters, t, L):
    """Oracle state after `iters` iterations: (s_prev, s, O, w) in the GPU's convention."""
    alg = Algorithm2(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, mu=1.0, t=t, schedule=L)
    s_prev = None
    for _ in range(iters):
        s_prev = alg.s.copy()
        alg.step()
    w = -alg.dual_multiplier()  # w = -mu y
    return alg, s_prev, alg.s.copy(), alg.O.copy(), w


PROBLEMS = {
    "cfg0": lambda: synth.config0(),
    "lp_powerlaw": lambda: synth.config1(scale=0.002),
    "socp": lambda: synth.config2(scale=0.002),
}


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert acs.lib().acs_init(0) == acs.ACS_OK, acs.lib().acs_last_error()


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("prec", [acs.PREC_FP64, acs.PREC_MIXED])
@pytest.mark.parametrize("l0", [57, 317])
@pytest.mark.parametrize("slices", [1, 8])
def test_one_iteration_parity(name, prec, l0, slices):
    p = PROBLEMS[name]()
    t, L = default_parameters(p.soc_sizes)
    alg, s_prev, s, O, w = _oracle_run(p, l0, t, L)
    if prec == acs.PREC_MIXED:
        s_prev, s = _f32(s_prev), _f32(s)
    st = acs.State(acs.Problem.from_synth(p), precision=prec, cg_max=2000,
                   cg_reduce=1e-13 if prec == acs.PREC_FP64 else 1e-7, a_slices=slices)
    st.set(l0, s_prev, s, O, w)
    st.step(1)
    g = st.get()
    ref = one_iteration(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, 1.0, s, O)
    errs = iterate_errors(g, ref, O)
    print(f"{name} prec={prec} l0={l0} slices={slices} (normwise/elementwise): {fmt(errs)}")
    assert g["l"] == l0 + 1
    assert np.array_equal(g["s_prev"], s)
    assert_iterate(errs, prec == acs.PREC_FP64, name)


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("prec", [acs.PREC_FP64, acs.PREC_MIXED])
@pytest.mark.parametrize("slices", [1, 8])
def test_conditioning_event_parity(name, prec, slices):
    p = PROBLEMS[name]()
    t, L = default_parameters(p.soc_sizes)
    l_event = L.first + L.every  # a member of L after the first event
    alg, s_prev, s, O, w = _oracle_run(p, l_event - 1, t, L)
    if prec == acs.PREC_MIXED:
        s_prev, s = _f32(s_prev), _f32(s)
    # oracle from exactly the shared state: x, z of the last iteration (steps 19-20)
    pp = abs_K(s_prev, p.n_orth, p.soc_sizes)
    alg.x = O * (pp + s) / 2.0
    alg.z = (pp - s) / (2.0 * O)
    alg.l = l_event - 1
    alg.step()  # conditions (steps 5-14) then iterates
    st = acs.State(acs.Problem.from_synth(p), precision=prec, cg_max=2000,
                   cg_reduce=1e-13 if prec == acs.PREC_FP64 else 1e-7, a_slices=slices)
    st.set(l_event - 1, s_prev, s, O, w)
    st.step(1)
    g = st.get()
    ref = {"O": alg.O, "s": alg.s, "x": alg.x, "z": alg.z}
    errs = iterate_errors(g, ref, alg.O, ("O", "s", "x", "z"))
    print(f"{name} prec={prec} slices={slices}: {fmt(errs)} O range {np.log(alg.O.max() / alg.O.min()):.3f}")
    assert_close({"O": errs.pop("O")}, 1e-9, name)
    assert_iterate(errs, prec == acs.PREC_FP64, name)


def _verify(p, x, y, z, info, eps):
    rec = kkt_errors(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, x, y, z)
    obj_err = _obj_err(rec["pobj"], p.p_star)
    print(f"{p.name}: status={info.status} iters={info.iterations} cg={info.cg_steps} gpu_kkt={info.kkt:.2e} "
          f"oracle_kkt={rec['kkt']:.2e} (p {rec['eps_p']:.1e} d {rec['eps_d']:.1e} g {rec['eps_g']:.1e} "
          f"k {rec['eps_k']:.1e}) eps_obj gpu {info.eps_obj:.2e} oracle {rec['eps_obj']:.2e} "
          f"obj_err={obj_err:.2e} solve_ms={info.solve_ms:.1f}")
    assert info.status == acs.SOLVED
    assert rec["kkt"] <= eps
    assert info.eps_obj <= eps / 1.05
    assert abs(info.eps_obj - rec["eps_obj"]) <= 1e-2 * eps
    return rec, obj_err


def test_solve_config0_fp64():
    p = synth.config0()
    x, y, z, info = acs.solve(acs.Problem.from_synth(p), precision=acs.PREC_FP64, eps_kkt=1e-6, max_iter=5000)
    rec, obj_err = _verify(p, x, y, z, info, 1.05e-6)
    assert obj_err <= 1e-5
    t, L = default_parameters(p.soc_sizes)
    alg = Algorithm2(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, mu=1.0, t=t, schedule=L)
    alg.run(5000, eps=1e-8, check_every=10)
    assert np.linalg.norm(z - alg.z) <= 1e-3 * (1 + np.linalg.norm(alg.z))
    assert np.linalg.norm(y - p.y0) <= 1e-3 * (1 + np.linalg.norm(p.y0))


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("slices", [1, 8])
def test_solve_mixed_to_1e4(name, slices):
    p = PROBLEMS[name]()
    x, y, z, info = acs.solve(acs.Problem.from_synth(p), precision=acs.PREC_MIXED, eps_kkt=1e-4, max_iter=20000,
                              a_slices=slices)
    rec, obj_err = _verify(p, x, y, z, info, 1.05e-4)
    assert obj_err <= 1e-4


def test_paper_example_fp64():
    import json
    import os

    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_example.json")))
    A = np.array(g["A"])
    rp = np.array([0, 5, 10, 15])
    prob = acs.Problem(3, 5, rp, np.tile(np.arange(5), 3), A.ravel(), np.array(g["b"]), np.array(g["c"]), 5)
    x, y, z, info = acs.solve(prob, precision=acs.PREC_FP64, eps_kkt=1e-8, check_every=1, auto_params=0, t=9.2,
                              l_first=1, l_every=1, l_last=50, max_iter=2000, cg_reduce=1e-14, cg_max=20)
    from tests._brute import lp_vertex_optimum

    best = lp_vertex_optimum(A, np.array(g["b"]), np.array(g["c"]))
    print(info.as_dict())
    assert info.status == acs.SOLVED
    assert abs(info.pobj - best[0]) <= 1e-6 * abs(best[0])
    assert np.allclose(x, best[2], atol=1e-5)


@pytest.mark.parametrize("cg_max", [1, 2, 3])
def test_cg_step_cap_both_layouts(cg_max):
    """A CG stopped by its step cap in every outer iteration (a reduction no
    step reaches): every iteration counts exactly cg_max steps with either
    layout (the one-slice CG finalizes its last step in a kernel of its own),
    and the two layouts' FP64 iterates agree to rounding after 1 and 20
    iterations."""
    p = synth.config1(scale=0.002)
    prob = acs.Problem.from_synth(p)
    outs = {}
    for slices in (1, 8):
        st = acs.State(prob, precision=acs.PREC_FP64, cg_max=cg_max, cg_reduce=1e-30, a_slices=slices)
        st.step(1)
        g1, c1 = st.get(), st.info().cg_steps
        st.step(19)
        g20, c20 = st.get(), st.info().cg_steps
        st.close()
        assert (c1, c20) == (cg_max, 20 * cg_max), (slices, c1, c20)
        outs[slices] = (g1, g20)
    for k, (a, b) in enumerate(zip(outs[1], outs[8])):
        for key in ("s", "w", "x", "z"):
            err = np.linalg.norm(a[key] - b[key]) / max(np.linalg.norm(b[key]), 1e-300)
            print(f"cg_max={cg_max} after {(1, 20)[k]}: {key} {err:.1e}")
            assert err <= 1e-9, (key, err)


def test_constraint_matrix_without_nonzeros():
    """A = 0 (m = 3 rows, no nonzeros), b = 0, c >= 0 on the orthant: the
    optimum is x = 0, z = c, objective 0, which the oracle reaches too.  Every
    product sweep then runs over empty rows (one-instance path, both layouts
    and precisions, and the batch kernel)."""
    m, n = 3, 5
    c = np.array([1.0, 2.0, 0.5, 0.0, 3.0])
    rp, ci, v, b = np.zeros(m + 1, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0), np.zeros(m)
    A = sp.csr_matrix((m, n))
    t, L = default_parameters([])
    alg = Algorithm2(A, b, c, n, [], mu=1.0, t=t, schedule=L)
    alg.run(2000, eps=1e-8, check_every=10)
    assert np.allclose(alg.x, 0.0) and np.allclose(alg.z, c)
    h = acs.Problem(m, n, rp, ci, v, b, c, n)
    for prec in (acs.PREC_FP64, acs.PREC_MIXED):
        for slices in (1, 8):
            x, y, z, info = acs.solve(h, precision=prec, eps_kkt=1e-8, max_iter=2000, a_slices=slices)
            assert info.status == acs.SOLVED, (prec, slices, info.status)
            tol = 1e-12 if prec == acs.PREC_FP64 else 1e-6
            assert np.abs(x).max() <= tol and np.abs(z - c).max() <= tol * np.abs(c).max(), (prec, slices)
            assert abs(info.pobj) <= tol
    bt = acs.Batch([h, h], eps_kkt=1e-8, max_iter=2000)
    bt.run(2000)
    for i in range(2):
        x, y, z, info = bt.result(i)
        assert info.status == acs.SOLVED and np.abs(x).max() <= 1e-6 and np.abs(z - c).max() <= 1e-6 * np.abs(c).max()
    bt.close()
    h.close()


@pytest.mark.parametrize("slices", [1, 8])
def test_determinism_bitwise(slices):
    p = synth.config1(scale=0.002)
    prob = acs.Problem.from_synth(p)
    outs = []
    for _ in range(2):
        st = acs.State(prob, precision=acs.PREC_MIXED, a_slices=slices)
        st.step(120)
        outs.append(st.get())
        st.close()
    for k in ("s", "s_prev", "O", "w", "x", "y", "z"):
        assert np.array_equal(outs[0][k], outs[1][k]), k


@pytest.mark.parametrize("name", ["cfg0", "socp"])
def test_solve_device_matches_solve_on_a_torch_stream(name):
    """acs_solve_device writes x, y, z into torch-allocated device tensors on
    torch's current (non-default) stream: bitwise the host-output solve."""
    import torch

    p = PROBLEMS[name]()
    prob = acs.Problem.from_synth(p)
    x, y, z, info = acs.solve(prob, eps_kkt=1e-4, max_iter=20000)
    dev = torch.device("cuda:0")
    s = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(s):
        xd = torch.full((p.n,), float("nan"), dtype=torch.float64, device=dev)
        yd = torch.full((p.m,), float("nan"), dtype=torch.float64, device=dev)
        zd = torch.full((p.n,), float("nan"), dtype=torch.float64, device=dev)
        info_d = acs.solve_device(prob, xd.data_ptr(), yd.data_ptr(), zd.data_ptr(), stream=s.cuda_stream,
                                  eps_kkt=1e-4, max_iter=20000)
        # a later torch op on the same stream sees the outputs
        total = float((xd.sum() + yd.sum() + zd.sum()).item())
    s.synchronize()
    assert info_d.status == info.status == acs.SOLVED
    assert info_d.iterations == info.iterations and info_d.pobj == info.pobj
    assert np.array_equal(xd.cpu().numpy(), x)
    assert np.array_equal(yd.cpu().numpy(), y)
    assert np.array_equal(zd.cpu().numpy(), z)
    assert np.isfinite(total)
    # a host pointer is refused before any GPU work
    host = np.zeros(p.n)
    with pytest.raises(acs.AcsError) as e:
        acs.solve_device(prob, host.ctypes.data, 0, 0)
    assert e.value.code == acs.ACS_ERR_ARG
