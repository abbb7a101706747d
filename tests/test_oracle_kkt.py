"""Pins of the oracle's KKT terms and objective-error estimate away from the
optimum: every term is checked against a value fixed by construction or by a
closed form, at points that are not optimal (a planted optimum makes every
term zero and pins nothing about its magnitude)."""
import math

import numpy as np
import scipy.sparse as sp

from oracle.cones import dist_K, proj_K
from oracle.kkt import kkt_errors, objective_bounds
from paper_2103_00736_amd import synth


def test_cone_distance_closed_forms():
    # orthant: distance is the norm of the negative part
    assert dist_K(np.array([-3.0, 4.0, -4.0]), 3, []) == 5.0
    # Lorentz cone, outside both the cone and its polar: |v0 - ||vbar||| / sqrt(2)
    assert math.isclose(dist_K(np.array([0.0, 3.0, 4.0]), 0, [3]), 5.0 / math.sqrt(2.0), rel_tol=1e-15)
    assert math.isclose(dist_K(np.array([1.0, 0.0, 6.0]), 0, [3]), 5.0 / math.sqrt(2.0), rel_tol=1e-15)
    # in the polar cone (||vbar|| <= -v0): the distance is ||v||
    assert math.isclose(dist_K(np.array([-5.0, 3.0, 0.0]), 0, [3]), math.sqrt(34.0), rel_tol=1e-15)
    # inside: zero; a product of the three cases adds in quadrature
    assert dist_K(np.array([5.0, 3.0, 4.0]), 0, [3]) == 0.0
    v = np.array([-2.0, 0.0, 3.0, 4.0, -5.0, 3.0, 0.0])
    assert math.isclose(dist_K(v, 1, [3, 3]), math.sqrt(4.0 + 12.5 + 34.0), rel_tol=1e-15)


def test_kkt_terms_at_a_constructed_point():
    """x, y, z chosen freely; b and c built so that A x - b = r_p and
    A^T y + z - c = r_d are known vectors; every term then has a closed form."""
    A = sp.csr_matrix(np.array([[1.0, 2.0, 0.0, -1.0, 0.5],
                                [0.0, -1.0, 3.0, 0.0, 2.0]]))
    x = np.array([2.0, -1.0, 0.0, 3.0, 4.0])  # orthant coordinate 1 is -1: dist 1; cone (0, 3, 4): dist 5/sqrt2
    z = np.array([0.5, 1.0, 6.0, 3.0, 4.0])   # cone (6, 3, 4) inside: dist 0
    y = np.array([1.0, -2.0])
    rp = np.array([0.3, -0.4])
    rd = np.array([1.0, 0.0, -2.0, 2.0, 0.0])
    b = A @ x - rp
    c = A.T @ y + z - rd
    rec = kkt_errors(A, b, c, 2, [3], x, y, z)
    assert math.isclose(rec["eps_p"], 0.5 / (1.0 + np.linalg.norm(b)), rel_tol=1e-14)
    assert math.isclose(rec["eps_d"], 3.0 / (1.0 + np.linalg.norm(c)), rel_tol=1e-14)
    pobj, dobj = float(c @ x), float(b @ y)
    assert math.isclose(rec["eps_g"], abs(pobj - dobj) / (1 + abs(pobj) + abs(dobj)), rel_tol=1e-14)
    dist_x = math.sqrt(1.0 + 12.5)
    assert math.isclose(rec["eps_k"], dist_x / (1.0 + max(np.linalg.norm(x), np.linalg.norm(z))), rel_tol=1e-14)
    # objective estimate: orthant |2 * 0.5| + |-1 * 1| = 2, cone |(0,3,4).(6,3,4)| = 25,
    # rows |0.3 * 1 + (-0.4) * (-2)| = 1.1
    assert math.isclose(rec["eps_obj"], (2.0 + 25.0 + 1.1) / (1.0 + abs(pobj)), rel_tol=1e-14)
    # it bounds the weak-duality form |c^T x - b^T y + r_d^T x| = |x^T z + y^T r_p| and |y^T r_p|
    gap_plus = pobj - dobj + float(rd @ x)
    assert abs(gap_plus) <= rec["eps_obj"] * (1.0 + abs(pobj)) and 1.1 <= rec["eps_obj"] * (1.0 + abs(pobj))
    # the identity the estimate rests on: c^T x - b^T y = z^T x - r_d^T x + r_p^T y
    assert math.isclose(pobj - dobj, float(z @ x - rd @ x + rp @ y), rel_tol=1e-14)


def test_objective_estimate_sums_lorentz_cones_with_signs():
    """Two Lorentz cones whose x_C^T z_C are +25 and -7 contribute |25 - 7|;
    orthant coordinates with products +3 and -2 contribute 3 + 2."""
    A = sp.csr_matrix(np.array([[1.0, 0.0, 2.0, 0.0, -1.0, 0.0, 1.0, 0.5]]))
    x = np.array([3.0, -1.0, 0.0, 3.0, 4.0, 1.0, 2.0, 2.0])
    z = np.array([1.0, 2.0, 6.0, 3.0, 4.0, 1.0, -2.0, -2.0])  # cone 2: 1 - 4 - 4 = -7
    y = np.array([2.0])
    rp = np.array([0.25])
    b = A @ x - rp
    c = A.T @ y + z
    rec = kkt_errors(A, b, c, 2, [3, 3], x, y, z)
    pobj = float(c @ x)
    assert math.isclose(rec["eps_obj"], (3.0 + 2.0 + 18.0 + 0.5) / (1.0 + abs(pobj)), rel_tol=1e-14)


def test_objective_bounds_hold_exactly_on_the_cone():
    """For x, z in K and a planted optimum (x0, y0, z0): y0^T r_p <= c^T x - p*
    <= c^T x - b^T y + r_d^T x0, whatever y; and the estimate eps_obj is within
    second-order terms of the true relative error near the optimum."""
    for p in (synth.lp_uniform(40, 100, 600, 17), synth.socp_percol(30, 90, 3, 5, 3, 8, 0.7)):
        A = p.scipy_csr()
        rng = np.random.default_rng(3)
        for scale in (1e-1, 1e-3, 1e-5):
            x = proj_K(p.x0 + scale * rng.standard_normal(p.n), p.n_orth, p.soc_sizes)
            z = proj_K(p.z0 + scale * rng.standard_normal(p.n), p.n_orth, p.soc_sizes)
            y = p.y0 + scale * rng.standard_normal(p.m)
            lo, hi = objective_bounds(A, p.b, p.c, x, y, z, p.x0, p.y0)
            err = float(p.c @ x) - p.p_star
            tol = 1e-12 * (1 + abs(p.p_star))
            assert lo - tol <= err <= hi + tol, (p.name, scale, lo, err, hi)
            rec = kkt_errors(A, p.b, p.c, p.n_orth, p.soc_sizes, x, y, z)
            true_rel = abs(err) / (1 + abs(rec["pobj"]))
            # at the optimum's own (y*, z*) the estimate is an exact bound for x in K
            star = kkt_errors(A, p.b, p.c, p.n_orth, p.soc_sizes, x, p.y0, p.z0)
            assert true_rel <= star["eps_obj"] * (1 + 1e-12) + 1e-15, (p.name, scale)
            # second-order slack: products of two perturbations of size `scale`
            assert true_rel <= rec["eps_obj"] + 50 * scale * scale * (1 + p.n), (p.name, scale)
