"""Pins of the oracle's Sinkhorn-Knopp equilibration and of Algorithm 2 on the
preconditioned problem (Sec. III: A_hat = D A E, b_hat = D b, c_hat = E c,
x_hat = E^{-1} x, z_hat = E z).

What fixes the equilibration without the oracle itself: the balance it is
defined to reach (unit row norms, column norms sqrt(m/n), a mean on every
Lorentz cone), a rank-one matrix whose balanced form is known in closed form
after one sweep, equivariance under permutations, and the rule for empty rows
and columns.  What fixes the preconditioned run: the paper's own printed
factors D^SK, E^SK with the printed condition number and the vertex optimum
of the worked example, planted optima, and the identity of the scaled run
with Algorithm 2 under the column scaling E O_hat.

Parity unpinned: the paper's D^SK, E^SK come from a regularized variant whose
regularization is not stated; the plain balancing does not reproduce them.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.alg2 import NO_CONDITIONING, Algorithm2, Schedule, conditioning_ratio, default_parameters, one_iteration
from oracle.equilibrate import EquilibratedAlgorithm2, sinkhorn_knopp_l2
from paper_2103_00736_amd import synth
from tests._brute import lp_vertex_optimum

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_example.json")


def _rand(m, n, density, seed):
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=density, random_state=rng, data_rvs=rng.standard_normal, format="csr")
    # every row and column nonzero (total support for the balance to exist)
    A = A + sp.csr_matrix((rng.standard_normal(m), (np.arange(m), rng.integers(0, n, m))), shape=(m, n))
    A = A + sp.csr_matrix((rng.standard_normal(n), (rng.integers(0, m, n), np.arange(n))), shape=(m, n))
    return sp.csr_matrix(A)


def _norms(A, d, e):
    B = (sp.diags(d) @ A @ sp.diags(e)).toarray()
    return np.linalg.norm(B, axis=1), np.linalg.norm(B, axis=0)


def test_balance_reached_at_convergence():
    A = _rand(30, 70, 0.2, 1)
    d, e = sinkhorn_knopp_l2(A, 70, [], 400)
    rn, cn = _norms(A, d, e)
    assert np.allclose(rn, 1.0, atol=1e-10)
    assert np.allclose(cn, np.sqrt(30 / 70), atol=1e-8)


def test_rank_one_balanced_after_one_sweep():
    """S = (u^2)(v^2)^T: the first sweep gives u'_i = 1/(u_i^2 V), V = sum v_j^2,
    then v'_j = V/(n v_j^2), so every entry of D A E has magnitude 1/sqrt(n)."""
    rng = np.random.default_rng(2)
    u, v = rng.uniform(0.1, 10, 7) * rng.choice([-1, 1], 7), rng.uniform(0.01, 100, 11) * rng.choice([-1, 1], 11)
    A = sp.csr_matrix(np.outer(u, v))
    for sweeps in (1, 5):
        d, e = sinkhorn_knopp_l2(A, 11, [], sweeps)
        B = (sp.diags(d) @ A @ sp.diags(e)).toarray()
        assert np.allclose(np.abs(B), 1.0 / np.sqrt(11), rtol=1e-12)
    d, e = sinkhorn_knopp_l2(A, 11, [], 1)
    V = float((v ** 2).sum())
    assert np.allclose(d, 1.0 / (np.abs(u) * np.sqrt(V)), rtol=1e-13)
    assert np.allclose(e, np.sqrt(V / 11) / np.abs(v), rtol=1e-13)


def test_lorentz_blocks_get_one_scale_and_mean_norm():
    rng = np.random.default_rng(3)
    cones = [4, 3, 6]
    n_orth = 9
    n = n_orth + sum(cones)
    A = _rand(12, n, 0.4, 4)
    d, e = sinkhorn_knopp_l2(A, n_orth, cones, 600)
    rn, cn = _norms(A, d, e)
    assert np.allclose(rn, 1.0, atol=1e-9)
    assert np.allclose(cn[:n_orth], np.sqrt(12 / n), atol=1e-8)
    off = n_orth
    for k in cones:
        blk = e[off:off + k]
        assert np.all(blk == blk[0])
        assert np.isclose(np.mean(cn[off:off + k] ** 2), 12 / n, atol=1e-8)
        off += k


def test_permutation_equivariant():
    A = _rand(15, 40, 0.3, 5)
    rng = np.random.default_rng(6)
    P, Q = rng.permutation(15), rng.permutation(40)
    d, e = sinkhorn_knopp_l2(A, 40, [], 25)
    dp, ep = sinkhorn_knopp_l2(A[P][:, Q], 40, [], 25)
    assert np.allclose(dp, d[P], rtol=1e-12) and np.allclose(ep, e[Q], rtol=1e-12)


def test_empty_rows_and_columns_keep_unit_scale():
    A = _rand(10, 20, 0.4, 7).tolil()
    A[3, :] = 0
    A[:, 5] = 0
    A[:, 11] = 0
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    d, e = sinkhorn_knopp_l2(A, 20, [], 300)
    assert d[3] == 1.0 and e[5] == 1.0 and e[11] == 1.0
    rn, cn = _norms(A, d, e)
    live_r = np.array([i != 3 for i in range(10)])
    assert np.allclose(rn[live_r], 1.0, atol=1e-8)


def test_paper_example_printed_factors():
    """The worked example of Sec. III with its printed D^SK, E^SK: the scaled
    matrix has the printed condition number, and Algorithm 1 on the
    preconditioned problem, mapped back, reaches the vertex optimum."""
    g = json.load(open(GOLD))
    A, b, c = sp.csr_matrix(np.array(g["A"])), np.array(g["b"]), np.array(g["c"])
    d, e = np.array(g["D_SK"]), np.array(g["E_SK"])
    sv = np.linalg.svd((sp.diags(d) @ A @ sp.diags(e)).toarray(), compute_uv=False)
    # the factors are printed to four digits: the condition number agrees to 1e-3
    assert abs(sv[0] / sv[-1] - g["cond_A_SK"]) / g["cond_A_SK"] < 1e-3
    best = lp_vertex_optimum(A.toarray(), b, c)
    alg = EquilibratedAlgorithm2(A, b, c, 5, [], d, e, mu=1.0, t=9.2, schedule=NO_CONDITIONING)
    for _ in range(6000):
        alg.step()
        if alg.l % 50 == 0 and alg.kkt()["kkt"] <= 1e-8:
            break
    rec = alg.kkt()
    assert rec["kkt"] <= 1e-8
    assert abs(rec["pobj"] - best[0]) <= 1e-6 * abs(best[0])
    assert np.allclose(alg.x, best[2], atol=1e-6)


@pytest.mark.parametrize("kind", ["lp", "socp"])
def test_scaled_run_is_algorithm2_with_scaling_E_times_O(kind):
    """One step of the scaled run from its state (s, O_hat) equals the
    original problem's step with the column scaling E O_hat (the row scaling D
    changes neither range((D A E O_hat)^T) nor the affine set), and the ratio
    of steps 5-10 taken from x_hat, z_hat is the original ratio over E^2."""
    if kind == "lp":
        p = synth.lp_uniform(40, 100, 400, 11)
    else:
        p = synth.socp_percol(40, 120, 3, 12, 3, 8, 0.7)
    A = p.scipy_csr()
    d, e = sinkhorn_knopp_l2(A, p.n_orth, p.soc_sizes, 20)
    t, _ = default_parameters(p.soc_sizes)
    alg = EquilibratedAlgorithm2(A, p.b, p.c, p.n_orth, p.soc_sizes, d, e, t=t, schedule=Schedule(1, 9, 40))
    for _ in range(30):
        alg.step()
    s, O = alg.s.copy(), alg.O.copy()
    ref = one_iteration(A, p.b, p.c, p.n_orth, p.soc_sizes, 1.0, s, O)
    alg.step()
    assert np.allclose(alg.s, ref["s"], rtol=0, atol=1e-10 * np.abs(ref["s"]).max())
    assert np.allclose(alg.x, ref["x"], rtol=0, atol=1e-10 * np.abs(ref["x"]).max())
    o_hat = conditioning_ratio(alg.inner.x, alg.inner.z, p.n_orth, p.soc_sizes)
    o = conditioning_ratio(alg.x, alg.z, p.n_orth, p.soc_sizes)
    fin = np.isfinite(o) & (o > 0)  # per coordinate, constant on every cone, as E is
    assert fin.sum() > 0.9 * p.n
    assert np.allclose(o_hat[fin], o[fin] / e[fin] ** 2, rtol=1e-10)


@pytest.mark.parametrize("kind", ["lp", "socp"])
def test_equilibrated_solve_reaches_planted_optimum(kind):
    if kind == "lp":
        p = synth.config1(scale=0.0004)
    else:
        p = synth.config2(scale=0.0004)
    A = p.scipy_csr()
    d, e = sinkhorn_knopp_l2(A, p.n_orth, p.soc_sizes, 25)
    t, L = default_parameters(p.soc_sizes)
    alg = EquilibratedAlgorithm2(A, p.b, p.c, p.n_orth, p.soc_sizes, d, e, t=t, schedule=L)
    rec = None
    while alg.l < 6000:
        alg.step()
        if alg.l % 20 == 0:
            rec = alg.kkt()
            if rec["kkt"] <= 1e-6:
                break
    assert rec["kkt"] <= 1e-6
    assert abs(rec["pobj"] - p.p_star) <= 1e-5 * (1 + abs(p.p_star))
    # the same problem without preconditioning reaches the same optimum
    plain = Algorithm2(A, p.b, p.c, p.n_orth, p.soc_sizes, t=t, schedule=L).run(6000, eps=1e-6, check_every=20)
    assert abs(plain["pobj"] - rec["pobj"]) <= 1e-5 * (1 + abs(p.p_star))
