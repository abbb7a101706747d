"""GPU tests of the persistent batched solver (acs_batch_*): every instance's
KKT error recomputed by the FP64 oracle, objectives against the planted
optimum and the one-instance solver, resumable runs and HIP-graph replays
bitwise equal to one eager run, and the lanes-per-row autotuner."""
import numpy as np
import pytest

from oracle.alg2 import Algorithm2, default_parameters
from oracle.cones import e_K
from oracle.kkt import kkt_errors
from paper_2103_00736_amd import acs, synth
from tests._parity import assert_close, errors, fmt, obj_err as _obj_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert acs.lib().acs_init(0) == acs.ACS_OK, acs.lib().acs_last_error()


def _mixed_set(k=24):
    """Uneven small LPs of the batch recipe (smaller m to keep the oracle quick)
    plus small SOCPs, and degenerate shapes (1-row, empty rows/columns)."""
    probs = []
    sizes = np.random.default_rng(5).integers(50, 400, size=k)
    for i, m in enumerate(sizes):
        probs.append(synth.config3(i, m=int(m)))
    for i in range(4):
        probs.append(synth.socp_percol(60 + 20 * i, 200 + 50 * i, 3, 100 + i, 3, 12, 0.8, name=f"socp{i}"))
    probs.append(synth.lp_uniform(1, 4, 3, 7, name="one_row"))
    probs.append(synth.lp_uniform(50, 125, 62, 8, name="sparse_empty"))
    return probs


def test_batch_matches_oracle_and_single_solver():
    probs = _mixed_set()
    handles = [acs.Problem.from_synth(p) for p in probs]
    b = acs.Batch(handles, eps_kkt=1e-4, max_iter=20000)
    ms = b.run(20000)
    print(f"batch of {len(probs)}: {ms:.1f} ms")
    for i, p in enumerate(probs):
        x, y, z, info = b.result(i)
        rec = kkt_errors(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, x, y, z)
        obj_err = _obj_err(rec["pobj"], p.p_star)
        print(f"  {p.name}: status={info.status} it={info.iterations} gpu_kkt={info.kkt:.2e} "
              f"oracle_kkt={rec['kkt']:.2e} eps_obj={info.eps_obj:.1e} obj_err={obj_err:.1e}")
        assert info.status == acs.SOLVED, p.name
        assert rec["kkt"] <= 1.05e-4, p.name
        assert abs(info.kkt - rec["kkt"]) <= 1e-6 + 1e-2 * rec["kkt"]
        assert obj_err <= 1e-4, p.name
    # alone (one-instance kernels) vs in the batch: both within 1e-4 of the optimum
    for i in (0, 5, len(probs) - 3):
        p = probs[i]
        x1, y1, z1, info1 = acs.solve(handles[i], eps_kkt=1e-4)
        _, _, _, info2 = b.result(i)
        assert _obj_err(info1.pobj, p.p_star) <= 1e-4 and _obj_err(info2.pobj, p.p_star) <= 1e-4


def test_resume_and_graph_replays_are_bitwise_equal():
    probs = [synth.config3(i, m=int(m)) for i, m in enumerate([300, 120, 80, 200, 60, 150])]
    handles = [acs.Problem.from_synth(p) for p in probs]
    ref = acs.Batch(handles, max_iter=3000)
    ref.run(3000, use_graph=False)
    chunks = acs.Batch(handles, max_iter=3000)
    for rep in range(60):  # graph replays with host work and syncs in between
        chunks.run(50, use_graph=True)
        _ = chunks.result(rep % len(probs))
    eager = acs.Batch(handles, max_iter=3000)
    for _ in range(60):
        eager.run(50, use_graph=False)
    for i in range(len(probs)):
        a, b_, c = ref.result(i), chunks.result(i), eager.result(i)
        for k in range(3):
            assert np.array_equal(a[k], b_[k]), (i, k)
            assert np.array_equal(a[k], c[k]), (i, k)
        assert a[3].iterations == b_[3].iterations == c[3].iterations


def test_autotune_and_cache(tmp_path):
    probs = [synth.config3(i, m=int(m)) for i, m in enumerate([400, 420, 60, 70, 1000])]
    handles = [acs.Problem.from_synth(p) for p in probs]
    cache = str(tmp_path / "tune.txt")
    b = acs.Batch(handles, max_iter=5000)
    b.autotune(sample=2, iters=10, cache_path=cache)
    lanes = [b.lanes(i) for i in range(len(probs))]
    assert all(g in (1, 2, 4, 8, 16, 32, 64, -512, -1024) for pair in lanes for g in pair)
    text = open(cache).read()
    assert text.startswith("gfx950")
    b.run(5000)
    for i, p in enumerate(probs):
        x, y, z, info = b.result(i)
        rec = kkt_errors(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, x, y, z)
        assert info.status == acs.SOLVED and rec["kkt"] <= 1.05e-4
    b2 = acs.Batch(handles, max_iter=5000)
    b2.autotune(sample=2, iters=10, cache_path=cache)  # served from the cache
    assert [b2.lanes(i) for i in range(len(probs))] == lanes


def _long_row_lp():
    """A planted LP whose row 0 and column 0 are longer than the batch kernel's
    LDS stage (1024 nonzeros), so both sweeps take the whole-workgroup row path
    right after a workgroup reduction."""
    import scipy.sparse as sp

    rng = np.random.default_rng(17)
    m, n = 1200, 3000
    A = np.where(rng.random((m, n)) < 0.004, rng.standard_normal((m, n)), 0.0)
    A[0, :] = rng.standard_normal(n)
    A[:, 0] = rng.standard_normal(m)
    A = A.astype(np.float32).astype(np.float64)
    x0 = np.where(rng.random(n) < 0.3, rng.random(n) + 0.1, 0.0)
    z0 = np.where(x0 > 0, 0.0, rng.random(n) + 0.1)
    y0 = rng.standard_normal(m)
    C = sp.csr_matrix(A)
    return C, A @ x0, A.T @ y0 + z0, float((A.T @ y0 + z0) @ x0)


def test_batch_long_rows_after_reductions():
    C, b, c, p_star = _long_row_lp()
    m, n = C.shape
    h = acs.Problem(m, n, C.indptr, C.indices, C.data, b, c, n)
    small = [synth.config3(i, m=int(mm)) for i, mm in enumerate([80, 120])]
    handles = [h] + [acs.Problem.from_synth(p) for p in small]
    bt = acs.Batch(handles, eps_kkt=1e-4, max_iter=20000)
    bt.run(20000)
    x, y, z, info = bt.result(0)
    rec = kkt_errors(C, b, c, n, np.zeros(0, np.int32), x, y, z)
    print(f"long rows: status={info.status} it={info.iterations} oracle_kkt={rec['kkt']:.2e} pobj={rec['pobj']:.6f} "
          f"p*={p_star:.6f}")
    assert info.status == acs.SOLVED
    assert rec["kkt"] <= 1.05e-4
    assert _obj_err(rec["pobj"], p_star) <= 1e-4
    _, _, _, one = acs.solve(h, eps_kkt=1e-4)
    assert _obj_err(one.pobj, p_star) <= 1e-4


def test_initial_state_of_every_instance():
    """Every instance of a freshly created batch holds the initial state of
    Alg. 2 (x = z = e_K: s_prev = (1+mu) e_K, s = (1-mu) e_K, O = 1, w = 0,
    unit row norms) before the first launch, and one iteration leaves none of
    them NaN.  Regression test of an arena zero-fill that was not ordered
    before the per-instance uploads on the batch's stream."""
    probs = [synth.config3(i, m=int(m)) for i, m in
             enumerate(np.random.default_rng(9).integers(50, 300, size=96))]
    probs += [synth.socp_percol(60, 180, 3, 300 + i, 3, 12, 0.8, name=f"socp{i}") for i in range(4)]
    handles = [acs.Problem.from_synth(p) for p in probs]
    b = acs.Batch(handles, max_iter=20000)
    for i, p in enumerate(probs):
        st = b.state(i)
        e = e_K(p.n_orth, p.soc_sizes)
        assert st["l"] == 0
        assert np.array_equal(st["s_prev"], 2.0 * e), i
        assert np.array_equal(st["s"], 0.0 * e), i
        assert np.array_equal(st["O"], np.ones(p.n)), i
        assert np.array_equal(st["w"], np.zeros(p.m)), i
        assert np.array_equal(st["dsq"], np.ones(p.m)), i
    b.run(1)
    for i in range(len(probs)):
        _, _, _, info = b.result(i, xyz=False)
        assert info.status != acs.NUMERIC, i
        assert b.state(i)["l"] == 1


def _oracle_k(p, k):
    t, L = default_parameters(p.soc_sizes)
    alg = Algorithm2(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, mu=1.0, t=t, schedule=L)
    s_prev = None
    for _ in range(k):
        s_prev = alg.s.copy()
        alg.step()
    return alg, s_prev


K_PARITY = 20
TIGHT = dict(cg_reduce=1e-7, cg_max=4000, eps_kkt=1e-14, check_every=1000000)


def _k_parity_set():
    return [synth.config3(0, m=120), synth.config3(1, m=260), synth.socp_percol(80, 240, 3, 41, 3, 12, 0.8),
            synth.lp_uniform(50, 125, 62, 8, name="sparse_empty")]


def test_batch_k_iterations_match_oracle():
    """20 iterations of the persistent kernel from the initial state (the
    l = 1 conditioning included) against 20 iterations of the literal FP64
    oracle, mixed precision with a tight CG: s, s_prev, O, w at 1e-5."""
    probs = _k_parity_set()
    b = acs.Batch([acs.Problem.from_synth(p) for p in probs], max_iter=K_PARITY, **TIGHT)
    b.run(K_PARITY)
    for i, p in enumerate(probs):
        alg, s_prev = _oracle_k(p, K_PARITY)
        g = b.state(i)
        A = p.scipy_csr()
        ref = {"s": alg.s, "s_prev": s_prev, "O": alg.O, "w": -alg.dual_multiplier()}
        # w is unique only where A has full row rank (empty or dependent rows
        # leave it free on the null space of A^T); A^T w always is
        g["A^T w"], ref["A^T w"] = A.T @ g["w"], A.T @ ref["w"]
        keys = ["s", "s_prev", "O", "A^T w"]
        if np.linalg.matrix_rank(A.toarray()) == p.m:
            keys.append("w")
        errs = errors(g, ref, keys)
        print(f"{p.name}: l={g['l']} {fmt(errs)}")
        assert g["l"] == K_PARITY
        assert_close(errs, 1e-5, p.name)
