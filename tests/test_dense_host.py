"""Host-side checks of the dense path (no GPU): the paper's dense generators
(Sec. V-B LPs, Sec. V-D SOCPs), the oracle pinned on them against SciPy's
HiGHS LP solver, and validation of dense problems at the C ABI."""
import numpy as np
import pytest
from scipy.optimize import linprog

from oracle.alg2 import Algorithm2, default_parameters
from oracle.kkt import kkt_errors
from paper_2103_00736_amd import acs, synth


def test_generators_follow_the_recipes():
    p = synth.e3_lp(200)
    assert (p.m, p.n) == (160, 200) and p.n_orth == 200 and len(p.soc_sizes) == 0
    assert np.all(np.abs(p.A) <= 1.0) and np.array_equal(p.A, p.A.astype(np.float32).astype(np.float64))
    assert np.all(p.x_feas >= 0) and np.allclose(p.A @ p.x_feas, p.b)
    q = synth.e6_socp(203, 10)
    assert (q.m, q.n, q.n_orth) == (162, 203, 3) and np.all(q.soc_sizes == 10) and len(q.soc_sizes) == 20
    assert np.all((q.c >= 0) & (q.c <= 1))
    for k in range(len(q.soc_sizes)):  # strictly inside every Lorentz cone
        off = q.n_orth + 10 * k
        assert q.x_feas[off] > np.linalg.norm(q.x_feas[off + 1:off + 10])
    assert np.allclose(q.A @ q.x_feas, q.b)


@pytest.mark.parametrize("n", [100, 250])
def test_oracle_reaches_the_lp_optimum_of_highs(n):
    """The oracle (Algorithm 2 step by step) on the paper's dense random LP
    reaches the optimum that an independent simplex/IPM code finds."""
    p = synth.e3_lp(n)
    t, L = default_parameters(p.soc_sizes)
    alg = Algorithm2(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, mu=1.0, t=t, schedule=L)
    alg.run(20000, eps=1e-8, check_every=10)
    rec = kkt_errors(p.scipy_csr(), p.b, p.c, p.n_orth, p.soc_sizes, alg.x, alg.dual_multiplier(), alg.z)
    lp = linprog(p.c, A_eq=p.A, b_eq=p.b, bounds=(0, None), method="highs")
    assert lp.status == 0
    assert rec["kkt"] <= 1e-8
    assert abs(rec["pobj"] - lp.fun) <= 1e-7 * (1 + abs(lp.fun))


def test_dense_problem_validation():
    p = synth.e3_lp(64)
    h = acs.Problem.from_dense(p.A, p.b, p.c, p.n_orth)
    assert h.device_bytes() >= 4 * p.m * p.n and h.batch_device_bytes() == -1
    h.close()
    bad = p.A.copy()
    bad[3, 5] = np.nan
    with pytest.raises(acs.AcsError) as ei:
        acs.Problem.from_dense(bad, p.b, p.c, p.n_orth)
    assert ei.value.code == acs.ACS_ERR_ARG
    with pytest.raises(acs.AcsError):
        acs.Problem.from_dense(p.A, p.b[:-1], p.c, p.n_orth)
    with pytest.raises(acs.AcsError):
        acs.Problem.from_dense(p.A, p.b, p.c, p.n_orth - 1)  # cones do not cover n
    # values that are not float32 numbers are kept exactly (an FP32 low part)
    q = acs.Problem.from_dense(p.A + 1e-9, p.b, p.c, p.n_orth)
    assert q.device_bytes() >= 8 * p.m * p.n
