"""Pins of the oracle's cone operators (Definition 1) against facts that do
not depend on its closed form: Moreau's decomposition theorem, a generic
constrained minimiser, idempotence, and the norm/inner-product properties of
abs_K for a self-dual cone."""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle.cones import abs_K, blocks, dist_K, e_K, proj_K, proj_lorentz


def _in_lorentz(u, tol=1e-12):
    return u[0] >= np.linalg.norm(u[1:]) - tol * (1 + np.abs(u).max())


@pytest.mark.parametrize("k", [1, 2, 3, 5, 17, 64, 65])
def test_moreau_decomposition(k):
    # u = proj(v) iff u in K, u - v in K (K self-dual: v - u in the polar), u^T (u - v) = 0
    rng = np.random.default_rng(k)
    for _ in range(200):
        v = rng.standard_normal(k) * rng.choice([0.01, 1.0, 100.0])
        u = proj_lorentz(v)
        assert _in_lorentz(u)
        assert _in_lorentz(u - v)
        assert abs(u @ (u - v)) <= 1e-12 * (1 + v @ v)


def test_projection_matches_generic_minimiser():
    rng = np.random.default_rng(7)
    for k in (2, 3, 4):
        for _ in range(10):
            v = rng.standard_normal(k)
            cons = [{"type": "ineq", "fun": lambda u: u[0] - np.sqrt(u[1:] @ u[1:] + 1e-300)}]
            res = minimize(lambda u: 0.5 * np.sum((u - v) ** 2), x0=np.r_[np.linalg.norm(v) + 1.0, np.zeros(k - 1)],
                           constraints=cons, method="SLSQP", options={"ftol": 1e-14, "maxiter": 500})
            assert np.allclose(proj_lorentz(v), res.x, atol=1e-5)


def test_boundary_branches_agree():
    # ||v_bar|| = v0 (on the boundary) and ||v_bar|| = -v0 (on the negative boundary)
    v = np.array([5.0, 3.0, 4.0])
    assert np.allclose(proj_lorentz(v), v)
    assert np.allclose(proj_lorentz(-v), 0.0)
    assert np.allclose(proj_lorentz(np.array([0.0, 0.0, 0.0])), 0.0)
    # the third branch at its edges tends to the first two
    eps = 1e-9
    assert np.allclose(proj_lorentz(np.array([5.0 - eps, 3.0, 4.0])), [5.0, 3.0, 4.0], atol=1e-8)


def test_orthant_is_size_one_lorentz():
    rng = np.random.default_rng(1)
    v = rng.standard_normal(50)
    assert np.array_equal(proj_K(v, 50, []), np.maximum(v, 0))
    assert np.allclose(abs_K(v, 50, []), np.abs(v))  # the "absolute value" of Def. 1
    for j in range(10):
        assert np.allclose(proj_lorentz(v[j:j + 1]), max(v[j], 0.0))


def _mixed(rng):
    sizes = [3, 1, 7, 2, 40]
    return 11, sizes, 11 + sum(sizes)


def test_product_cone_properties():
    rng = np.random.default_rng(3)
    n_orth, sizes, n = _mixed(rng)
    for _ in range(50):
        v = rng.standard_normal(n) * 3
        u = proj_K(v, n_orth, sizes)
        assert np.allclose(proj_K(u, n_orth, sizes), u)  # idempotent
        a = abs_K(v, n_orth, sizes)
        assert np.isclose(np.linalg.norm(a), np.linalg.norm(v))  # norm preserved
        assert dist_K(a, n_orth, sizes) <= 1e-10 * np.linalg.norm(v)  # abs_K(v) in K
        # abs_K(v) = proj(v) + proj(-v) for a self-dual cone
        assert np.allclose(a, proj_K(v, n_orth, sizes) + proj_K(-v, n_orth, sizes))
        w = rng.standard_normal(n)
        assert abs_K(w, n_orth, sizes) @ a >= w @ v - 1e-10


def test_blocks_and_identity_layout():
    got = list(blocks(2, [3, 1]))
    assert got == [(0, 1), (1, 1), (2, 3), (5, 1)]
    e = e_K(2, [3, 1])
    assert np.array_equal(e, [1, 1, 1, 0, 0, 1])
    with pytest.raises(ValueError):
        proj_K(np.zeros(5), 2, [4])
