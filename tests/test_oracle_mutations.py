"""Plants plausible mistakes in the oracle (on the CPU) and checks that the
pin tests catch each one: a pin suite that passed on a wrong oracle would
not pin anything.  Each mutation replaces one oracle function for the
duration of the test; the pins are the functions of the other oracle test
modules, run as plain calls."""
import numpy as np
import pytest

import oracle.alg2 as alg2
import oracle.cones as cones
import oracle.equilibrate as equilibrate
import oracle.kkt as kkt
import oracle.subspace as subspace
from tests import test_oracle_alg2 as P2
from tests import test_oracle_cones as PC
from tests import test_oracle_equilibrate as PE
from tests import test_oracle_kkt as PK
from tests import test_oracle_subspace as PS

PINS = [
    lambda: PC.test_moreau_decomposition(3),
    lambda: PC.test_moreau_decomposition(17),
    PC.test_orthant_is_size_one_lorentz,
    PC.test_product_cone_properties,
    lambda: PS.test_projector_matches_numpy_pinv(0),
    PS.test_projector_algebra,
    PS.test_paper_example_condition_numbers,
    P2.test_ratio_worked_orthant,
    P2.test_ratio_worked_soc,
    P2.test_normalisation_within_range_is_identity_power,
    P2.test_normalisation_caps_log_range,
    P2.test_normalisation_guards,
    P2.test_lemma1_norm_and_inner_product,
    lambda: P2.test_lemma2_planted_fixed_point(1.0),
    P2.test_lemma2_in_any_scaling,
    P2.test_lemma3_monotone_distance,
    lambda: P2.test_algorithm1_is_douglas_rachford(True),
    P2.test_paper_example_reaches_vertex_optimum,
    P2.test_fused_update_identity,
    P2.test_kkt_at_planted_point_and_ls_multiplier,
    PK.test_cone_distance_closed_forms,
    PK.test_kkt_terms_at_a_constructed_point,
    PK.test_objective_bounds_hold_exactly_on_the_cone,
    PK.test_objective_estimate_sums_lorentz_cones_with_signs,
    PE.test_balance_reached_at_convergence,
    PE.test_rank_one_balanced_after_one_sweep,
    PE.test_lorentz_blocks_get_one_scale_and_mean_norm,
    PE.test_paper_example_printed_factors,
    lambda: PE.test_scaled_run_is_algorithm2_with_scaling_E_times_O("socp"),
]


def _caught():
    for pin in PINS:
        try:
            pin()
        except Exception:
            return True
    return False


def _mut_abs_dropped_term(v, n_orth, soc_sizes):
    return cones.proj_K(v, n_orth, soc_sizes)


def _mut_lorentz_scale(v):
    v = np.asarray(v, dtype=np.float64)
    nv = float(np.linalg.norm(v[1:]))
    if nv <= v[0]:
        return v.copy()
    if nv <= -v[0]:
        return np.zeros_like(v)
    a = v[0] + nv  # missing the factor 1/2
    out = np.empty_like(v)
    out[0] = a
    out[1:] = (a / nv) * v[1:]
    return out


def _mut_reflect(self, v):
    return self.project(v) - np.asarray(v)  # missing factor 2


def _mut_pinv_transposed(self, b):
    return self.B.T @ np.asarray(b)  # B^T b instead of B^T (B B^T)^+ b


def _mut_ratio_inverted(x, z, n_orth, soc_sizes):
    return alg2_orig_ratio(z, x, n_orth, soc_sizes)


def _mut_no_cap(o_raw, t):
    o = np.abs(np.asarray(o_raw, dtype=np.float64))
    o = np.where(np.isnan(o), 1.0, o)
    valid = np.isfinite(o) & (o > 0)
    if not valid.any():
        return np.ones_like(o)
    lo, hi = o[valid].min(), o[valid].max()
    o = np.where(o == 0, lo, np.where(np.isinf(o), hi, o))
    span = np.log(hi) - np.log(lo)
    return o ** (1.0 if span <= 0 else t / span)  # min(1, .) dropped


alg2_orig_ratio = alg2.conditioning_ratio
kkt_orig_errors = kkt.kkt_errors


def _mut_dist_squared(v, n_orth, soc_sizes):
    d = np.asarray(v, dtype=np.float64) - cones.proj_K(v, n_orth, soc_sizes)
    return float(d @ d)  # squared distance


def _mut_dual_residual_sign(A, b, c, n_orth, soc_sizes, x, y, z):
    return kkt_orig_errors(A, b, c, n_orth, soc_sizes, x, y, -np.asarray(z))  # A^T y - z - c


def _mut_objective_drops_rp(A, b, c, n_orth, soc_sizes, x, y, z):
    rec = kkt_orig_errors(A, b, c, n_orth, soc_sizes, x, y, z)
    x, z = np.asarray(x), np.asarray(z)
    xz = [abs(float(x[st:st + k] @ z[st:st + k])) for st, k in cones.blocks(n_orth, soc_sizes)]
    rec["eps_obj"] = float(np.sum(xz)) / (1 + abs(rec["pobj"]))  # without |y^T r_p|
    return rec


def _mut_objective_signed(A, b, c, n_orth, soc_sizes, x, y, z):
    rec = kkt_orig_errors(A, b, c, n_orth, soc_sizes, x, y, z)
    x, z, y = np.asarray(x), np.asarray(z), np.asarray(y)
    rp = A @ x - b
    rec["eps_obj"] = (abs(float(x @ z)) + abs(float(rp @ y))) / (1 + abs(rec["pobj"]))  # x^T z before |.|
    return rec


def _mut_objective_cones_absolute(A, b, c, n_orth, soc_sizes, x, y, z):
    rec = kkt_orig_errors(A, b, c, n_orth, soc_sizes, x, y, z)
    x, z, y = np.asarray(x), np.asarray(z), np.asarray(y)
    rp = A @ x - b
    xz = [abs(float(x[st:st + k] @ z[st:st + k])) for st, k in cones.blocks(n_orth, soc_sizes)]
    rec["eps_obj"] = (float(np.sum(xz)) + abs(float(rp @ y))) / (1 + abs(rec["pobj"]))  # |.| cone by cone
    return rec


def _mut_objective_bounds_sign(A, b, c, x, y, z, x_opt, y_opt):
    rp = A @ np.asarray(x) - b
    rd = A.T @ np.asarray(y) + np.asarray(z) - c
    gap = float(c @ x) - float(b @ y)
    return float(np.asarray(y_opt) @ rp), gap - float(rd @ np.asarray(x_opt))


def _patched_step(kind):
    orig = alg2.Algorithm2.step

    def step(self):
        self.l += 1
        if self.l in self.schedule:
            self.condition()
        s = self.s
        p = cones.abs_K(s, self.n_orth, self.soc_sizes)
        r = self.proj.reflect(p)
        if kind == "sign18":
            s_new = 0.5 * s + 0.5 * r + self.d
        else:
            s_new = 0.5 * s - 0.5 * r + self.d
        if kind == "x_without_O":
            self.x = (p + s_new) / 2.0
        else:
            self.x = self.O * (p + s_new) / 2.0
        self.z = (p - s_new) / (2.0 * self.mu * self.O)
        self.p = p
        self.s = s_new

    return step, orig


def _patched_condition_recast():
    def condition(self):
        o = alg2.conditioning_ratio(self.x, self.z, self.n_orth, self.soc_sizes)
        O = alg2.normalize_scaling(o, self.t)
        self.O = O
        self.proj = subspace.RangeProjector(self.A, O, method=self.method)
        Oc = O * self.c
        self.d = self.proj.pinv_apply(self.b) + 0.5 * self.mu * (self.proj.reflect(Oc) - Oc)
        self.s = self.x * O - self.mu * self.z / O  # step 14 with the scaling inverted

    return condition


def _patched_condition_no_pinv_b():
    def condition(self):
        o = alg2.conditioning_ratio(self.x, self.z, self.n_orth, self.soc_sizes)
        O = alg2.normalize_scaling(o, self.t)
        self.O = O
        self.proj = subspace.RangeProjector(self.A, O, method=self.method)
        Oc = O * self.c
        self.d = 0.5 * self.mu * (self.proj.reflect(Oc) - Oc)  # (AO)^dagger b dropped
        self.s = self.x / O - self.mu * O * self.z

    return condition


def _sk_variant(kind):
    """The equilibration with one planted mistake."""
    import scipy.sparse as sp

    def sk(A, n_orth, soc_sizes, sweeps):
        A = sp.csr_matrix(A, dtype=np.float64)
        m, n = A.shape
        S = abs(A) if kind == "abs" else A.multiply(A).tocsr()
        v, u = np.ones(n), np.ones(m)
        target = 1.0 if kind == "target" else m / n
        for _ in range(int(sweeps)):
            rs = S @ v
            u = np.where(rs > 0, 1.0 / np.where(rs > 0, rs, 1.0), 1.0)
            cs = S.T @ u
            for start, k in cones.blocks(n_orth, soc_sizes):
                if kind == "per_coordinate":
                    c = cs[start:start + k]
                    v[start:start + k] = np.where(c > 0, target / np.where(c > 0, c, 1.0), 1.0)
                else:
                    tot = float(cs[start:start + k].sum())
                    v[start:start + k] = target * k / tot if tot > 0 else 1.0
        return np.sqrt(u), np.sqrt(v)

    return sk


def _mut_z_mapped_with_e(self):
    return self.inner.z * self.e  # z = E^{-1} z_hat


MUTATIONS = {
    "abs_K returns proj_K": (cones, "abs_K", _mut_abs_dropped_term),
    "Lorentz projection scale": (cones, "proj_lorentz", _mut_lorentz_scale),
    "reflection without factor 2": (subspace.RangeProjector, "reflect", _mut_reflect),
    "pseudo-inverse without (BB^T)^+": (subspace.RangeProjector, "pinv_apply", _mut_pinv_transposed),
    "ratio inverted": (alg2, "conditioning_ratio", _mut_ratio_inverted),
    "exponent not capped at 1": (alg2, "normalize_scaling", _mut_no_cap),
    "step 18 sign": (alg2.Algorithm2, "step", _patched_step("sign18")[0]),
    "step 19 without O": (alg2.Algorithm2, "step", _patched_step("x_without_O")[0]),
    "step 14 scaling inverted": (alg2.Algorithm2, "condition", _patched_condition_recast()),
    "step 13 drops (AO)^dagger b": (alg2.Algorithm2, "condition", _patched_condition_no_pinv_b()),
    "cone distance squared": (cones, "dist_K", _mut_dist_squared),
    "dual residual with -z": (kkt, "kkt_errors", _mut_dual_residual_sign),
    "objective estimate without |y^T r_p|": (kkt, "kkt_errors", _mut_objective_drops_rp),
    "objective estimate summed before the absolute values": (kkt, "kkt_errors", _mut_objective_signed),
    "objective estimate with |x_C^T z_C| cone by cone": (kkt, "kkt_errors", _mut_objective_cones_absolute),
    "objective bound with -r_d": (kkt, "objective_bounds", _mut_objective_bounds_sign),
    "equilibration on |a| instead of a^2": (equilibrate, "sinkhorn_knopp_l2", _sk_variant("abs")),
    "equilibration column target 1": (equilibrate, "sinkhorn_knopp_l2", _sk_variant("target")),
    "equilibration per coordinate on cones": (equilibrate, "sinkhorn_knopp_l2", _sk_variant("per_coordinate")),
    "preconditioned z mapped back with E": (equilibrate.EquilibratedAlgorithm2, "z", property(_mut_z_mapped_with_e)),
}


def test_unmutated_oracle_passes_every_pin():
    assert not _caught()


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    target, attr, repl = MUTATIONS[name]
    monkeypatch.setattr(target, attr, repl)
    # modules that imported the name directly see the mutation too
    for mod in (alg2, kkt, subspace, P2, PC, PK, PS, PE):
        if hasattr(mod, attr) and mod is not target and callable(getattr(mod, attr)) and target in (
                cones, alg2, kkt, equilibrate):
            monkeypatch.setattr(mod, attr, repl)
    assert _caught(), f"no pin caught: {name}"
