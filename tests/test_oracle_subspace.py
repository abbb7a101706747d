"""Pins of the oracle's subspace reflection and pseudo-inverse against NumPy's
SVD-based pinv, the projector's algebraic properties, and the condition
numbers the paper prints for its worked example (which fix that the
conditioning multiplies A by O on the right)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.subspace import RangeProjector
from paper_2103_00736_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_example.json")


def _rand_sparse(m, n, density, seed, empty_rows=0):
    rng = np.random.default_rng(seed)
    A = sp.random(m, n, density=density, random_state=rng, data_rvs=rng.standard_normal, format="csr")
    A = A.tolil()
    for i in range(empty_rows):
        A[i, :] = 0
    return sp.csr_matrix(A)


@pytest.mark.parametrize("empty_rows", [0, 3])
def test_projector_matches_numpy_pinv(empty_rows):
    A = _rand_sparse(30, 80, 0.15, 11, empty_rows)
    O = np.exp(np.random.default_rng(2).uniform(-3, 3, 80))
    P = RangeProjector(A, O, method="exact")
    B = A.toarray() * O
    Bp = np.linalg.pinv(B)
    rng = np.random.default_rng(5)
    for _ in range(5):
        v = rng.standard_normal(80)
        assert np.allclose(P.project(v), Bp @ (B @ v), atol=1e-10)
        bb = B @ rng.standard_normal(80)
        assert np.allclose(P.pinv_apply(bb), Bp @ bb, atol=1e-10)


def test_projector_algebra():
    A = _rand_sparse(40, 100, 0.1, 21)
    O = np.exp(np.random.default_rng(1).uniform(-2, 2, 100))
    P = RangeProjector(A, O)
    B = A.toarray() * O
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal(100), rng.standard_normal(100)
    Pu = P.project(u)
    assert np.allclose(P.project(Pu), Pu, atol=1e-10)  # idempotent
    assert np.isclose(Pu @ v, u @ P.project(v))  # symmetric
    assert np.allclose(B @ Pu, B @ u, atol=1e-10)  # B P = B
    r = P.reflect(u)
    assert np.isclose(np.linalg.norm(r), np.linalg.norm(u))  # isometry
    assert np.allclose(P.reflect(r), u, atol=1e-10)  # involution


def test_pcg_matches_exact():
    p = synth.lp_uniform(300, 800, 4000, 99)
    A = p.scipy_csr()
    O = np.exp(np.random.default_rng(3).uniform(-1, 1, 800))
    Pe = RangeProjector(A, O, method="exact")
    Pc = RangeProjector(A, O, method="pcg")
    v = np.random.default_rng(4).standard_normal(800)
    assert np.allclose(Pe.project(v), Pc.project(v), atol=1e-8)
    assert np.allclose(Pe.pinv_apply(p.b), Pc.pinv_apply(p.b), atol=1e-8)


def test_paper_example_condition_numbers():
    g = json.load(open(GOLD))
    A = sp.csr_matrix(np.array(g["A"]))
    cond = lambda M: np.linalg.cond(M.toarray() if sp.issparse(M) else M)
    assert abs(cond(A) - g["cond_A"]) / g["cond_A"] < 1e-4
    # the oracle's scaled matrix A O (post-multiplication, D = I) reproduces the
    # printed condition number of the adaptively conditioned matrix
    B = RangeProjector(A, np.array(g["E_AC"])).B
    assert abs(cond(B) - g["cond_A_AC"]) / g["cond_A_AC"] < 1e-5
    # a pre-multiplied or inverted scaling does not
    assert abs(cond(A.toarray() / np.array(g["E_AC"])) - g["cond_A_AC"]) / g["cond_A_AC"] > 0.1
    # D A E with the printed Sinkhorn-Knopp factors (given to 3 significant figures)
    M = np.diag(g["D_SK"]) @ A.toarray() @ np.diag(g["E_SK"])
    assert abs(cond(M) - g["cond_A_SK"]) / g["cond_A_SK"] < 1e-3


@pytest.mark.parametrize("empty_rows", [0, 4])
def test_normal_pinv_penrose(empty_rows):
    """(B B^T)^+ satisfies the four Penrose conditions for G = B B^T and is
    zero on empty rows; on live rows it inverts G."""
    A = _rand_sparse(25, 60, 0.2, 31, empty_rows)
    O = np.exp(np.random.default_rng(7).uniform(-2, 2, 60))
    P = RangeProjector(A, O, method="exact")
    B = A.toarray() * O
    G = B @ B.T
    X = P.normal_pinv()
    sc = np.abs(X).max() * np.abs(G).max()
    assert np.abs(G @ X @ G - G).max() <= 1e-10 * np.abs(G).max()
    assert np.abs(X @ G @ X - X).max() <= 1e-10 * np.abs(X).max() * sc
    assert np.abs(X - X.T).max() <= 1e-12 * np.abs(X).max()
    assert np.abs(G @ X - (G @ X).T).max() <= 1e-10 * sc
    live = np.abs(B).sum(axis=1) > 0
    assert not X[~live].any() and not X[:, ~live].any()
    assert np.abs((G @ X)[np.ix_(live, live)] - np.eye(live.sum())).max() <= 1e-10 * sc


def test_normal_pinv_closed_forms():
    # rows with disjoint supports: G is diagonal, G_ii = sum_j a_ij^2 O_j^2
    A = sp.csr_matrix(np.array([[1.0, 2.0, 0, 0], [0, 0, 3.0, 0], [0, 0, 0, 0]]))
    O = np.array([0.5, 2.0, 1.0, 7.0])
    X = RangeProjector(A, O, method="exact").normal_pinv()
    assert np.allclose(X, np.diag([1 / (0.25 + 16.0), 1 / 9.0, 0.0]), rtol=1e-14, atol=0)
    # two rows: the 2 x 2 inverse by its cofactor formula
    A = sp.csr_matrix(np.array([[1.0, 1.0, 0.0], [1.0, -1.0, 2.0]]))
    O = np.array([1.0, 3.0, 0.5])
    g11, g12, g22 = 1 + 9, 1 - 9, 1 + 9 + 1
    det = g11 * g22 - g12 * g12
    want = np.array([[g22, -g12], [-g12, g11]]) / det
    assert np.allclose(RangeProjector(A, O, method="exact").normal_pinv(), want, rtol=1e-13, atol=0)
