"""Mutation check of the oracle's pins.

Each mutant plants one plausible mistake in the oracle (a sign flip, a
dropped term, a transposed factor, swapped operands, an exchanged order) and
the test asserts that at least one pin of tests/test_oracle_pins*.py then
fails.  Python mutants replace one function or constant of
``oracle/preprocess.py`` for the duration of the check; C mutants are copies
of ``oracle/raster.c`` with one expression changed, compiled with gcc into a
temporary directory and loaded in place of the oracle's library.  Nothing
here touches the GPU path.
"""
import math
import os
import subprocess

import numpy as np
import pytest
import torch

from oracle import build as obuild
from oracle import preprocess as pp
from oracle import raster

import test_oracle_pins as P
import test_oracle_pins_geometry as G

F64 = torch.float64

# every pin, with its parameters; run in this order, stopping at the first failure
PINS = [
    ("beta_map", P.test_beta_map_paper_values, {}),
    ("covariance_6_0", P.test_covariance_matches_appendix_blocks, {"dim": 6, "rot": 0}),
    ("covariance_7_1", P.test_covariance_matches_appendix_blocks, {"dim": 7, "rot": 1}),
    ("quat_orthonormal", P.test_quaternion_rotation_is_orthonormal, {}),
    ("skew", P.test_skew_rotation_first_order_properties, {}),
    ("cond_textbook_6", P.test_conditioning_is_textbook_gaussian_when_modulation_is_one, {"dim": 6}),
    ("cond_textbook_7", P.test_conditioning_is_textbook_gaussian_when_modulation_is_one, {"dim": 7}),
    ("cond_c1", P.test_conditioning_one_query_dimension_closed_form, {}),
    ("cond_diag", P.test_conditioning_diagonal_query_covariance_per_dimension_modulation, {}),
    ("cond_symmetric", P.test_conditioning_result_is_symmetric, {}),
    ("whitening", P.test_whitening_identity_and_factor, {}),
    ("chol_not_Lq", P.test_opacity_whitens_with_cholesky_of_sigma_q_not_L_q, {}),
    ("reduce_3d_7", P.test_zero_cross_correlation_and_flat_query_reduce_to_3d, {"dim": 7}),
    ("projection_jacobian", P.test_projection_matches_numerical_jacobian, {}),
    ("isotropic_closed_form", P.test_single_isotropic_primitive_closed_form, {"b_x": 0.0}),
    ("gaussian_limit", P.test_gaussian_limit_printed_bound, {}),
    ("conic_inverse", G.test_record_conic_is_inverse_of_projected_covariance, {"case": 0}),
    ("conic_pixels", G.test_anisotropic_splat_pixels_follow_the_mahalanobis_distance, {"case": 1}),
    ("camera_center", G.test_camera_center_is_where_the_camera_was_placed,
     {"center": (1.2, -0.5, -4.0)}),
    ("query_hand", G.test_query_direction_hand_values, {}),
    ("query_at_mean_6", G.test_query_at_the_primitive_mean_keeps_the_opacity, {"dim": 6}),
    ("query_at_mean_7", G.test_query_at_the_primitive_mean_keeps_the_opacity, {"dim": 7}),
    ("composite_brute", P.test_compositing_matches_product_form_brute_force, {}),
    ("composite_invariants", P.test_compositing_invariants, {}),
    ("early_termination", P.test_early_termination_golden, {}),
    ("binning_brute", P.test_binning_is_exact_and_complete_brute_force, {}),
    ("binning_keys", P.test_binning_keys_sort_and_ranges, {}),
    ("tile_threshold", P.test_tile_test_threshold_golden, {"a": 2.0, "b": 0.5, "c": 1.0}),
    ("opacity_clamp", P.test_opacity_clamp_golden, {}),
    ("stop_ends_pixel", P.test_stop_ends_the_pixel, {}),
    ("raster_adjoint_fd", P.test_raster_adjoint_matches_finite_differences_on_records,
     {"saturated": False}),
    ("raster_adjoint_fd_saturated", P.test_raster_adjoint_matches_finite_differences_on_records,
     {"saturated": True}),
    ("oracle_fd_7", P.test_oracle_gradient_matches_finite_differences,
     {"dim": 7, "rot": 0, "dist": "cfg3"}),
]


def _first_failing_pin():
    for name, fn, kw in PINS:
        try:
            fn(**kw)
        except Exception:   # an assertion, or a mutant that breaks the arithmetic outright
            return name
    return None


# ------------------------------------------------------------------ Python mutants
def _m_conic_swap_ac(mp):
    mp.setattr(pp, "conic", lambda Sp, det: (Sp[:, 0, 0] / det, -Sp[:, 0, 1] / det, Sp[:, 1, 1] / det))


def _m_conic_flip_b(mp):
    mp.setattr(pp, "conic", lambda Sp, det: (Sp[:, 1, 1] / det, Sp[:, 0, 1] / det, Sp[:, 0, 0] / det))


def _m_no_dilation(mp):
    mp.setattr(pp, "DILATION", 0.0)


def _m_camera_center_sign(mp):
    mp.setattr(pp, "camera_center", lambda view: torch.as_tensor(view.R, dtype=F64).T
               @ torch.as_tensor(view.t, dtype=F64))


def _m_query_reversed(mp):
    orig = pp.query

    def q(mu_x, view, C):
        out = orig(mu_x, view, C)
        if C == 3:
            return -out
        out = out.clone()
        out[:, 1:4] = -out[:, 1:4]
        return out
    mp.setattr(pp, "query", q)


def _m_query_order_dt(mp):
    orig = pp.query

    def q(mu_x, view, C):
        out = orig(mu_x, view, C)
        if C >= 4:
            out = torch.cat([out[:, 1:4], out[:, :1], out[:, 4:]], 1)
        return out
    mp.setattr(pp, "query", q)


def _modulated_opacity_variant(transpose_whitening=False, exponent_scale=4.0):
    def f(o, Sigma_q, v, b_q):
        if v.shape[1] == 0:
            return o
        Lhat = torch.linalg.cholesky(Sigma_q)
        if transpose_whitening:
            w = torch.linalg.solve_triangular(Lhat.transpose(-1, -2), v[:, :, None], upper=True)[:, :, 0]
        else:
            w = torch.linalg.solve_triangular(Lhat, v[:, :, None], upper=False)[:, :, 0]
        x = w * w
        log1md = math.log(2.0) - 2.0 * x - torch.log1p(torch.exp(-2.0 * x))
        return o * torch.exp((exponent_scale * torch.exp(b_q) * log1md).sum(dim=1))
    return f


def _m_whitening_transposed(mp):
    mp.setattr(pp, "modulated_opacity", _modulated_opacity_variant(transpose_whitening=True))


def _m_opacity_exponent(mp):
    mp.setattr(pp, "modulated_opacity", _modulated_opacity_variant(exponent_scale=1.0))


def _m_beta_map(mp):
    mp.setattr(pp, "beta_of_b", lambda b: torch.exp(b))


def _m_beta_tilde_max(mp):
    mp.setattr(pp, "beta_tilde", lambda b: torch.where(b > 0, torch.exp(torch.clamp(b, min=0.0)),
                                                      torch.ones_like(b)))


def _condition_variant(mean_sign=1.0, modulate_cov=True, symmetrise=True):
    def f(mu_x, Sigma, v, b_q, beta_modulated=True):
        C = v.shape[1]
        Sx = Sigma[:, :3, :3]
        if C == 0:
            return mu_x, Sx
        Sxq = Sigma[:, :3, 3:]
        Sq = Sigma[:, 3:, 3:]
        K = torch.linalg.solve(Sq, Sxq.transpose(-1, -2)).transpose(-1, -2)
        bt = pp.beta_tilde(b_q) if beta_modulated else torch.ones_like(b_q)
        KD = K @ torch.diag_embed(bt)
        mu_c = mu_x + mean_sign * (KD @ v[:, :, None])[:, :, 0]
        M = (KD if modulate_cov else K) @ Sxq.transpose(-1, -2)
        S_c = Sx - (0.5 * (M + M.transpose(-1, -2)) if symmetrise else M)
        return mu_c, S_c
    return f


def _m_condition_mean_sign(mp):
    mp.setattr(pp, "condition", _condition_variant(mean_sign=-1.0))


def _m_condition_cov_unmodulated(mp):
    mp.setattr(pp, "condition", _condition_variant(modulate_cov=False))


def _m_condition_not_symmetrised(mp):
    mp.setattr(pp, "condition", _condition_variant(symmetrise=False))


def _m_rotation_transposed(mp):
    orig = pp.rotation_matrix
    mp.setattr(pp, "rotation_matrix", lambda rp, rot: orig(rp, rot).transpose(-1, -2))


def _m_lqx_transposed(mp):
    orig = pp.lower_factor

    def f(fields, dim, rot):
        C = dim - 3
        if C == 3:
            fields = dict(fields)
            n = fields["L_qx"].shape[1]
            fields["L_qx"] = fields["L_qx"].T.reshape(n, 3, 3).transpose(1, 2).reshape(n, 9).T
        return orig(fields, dim, rot)
    mp.setattr(pp, "lower_factor", f)


def _m_jacobian_no_depth_term(mp):
    def project(mu_c, S_c, view):
        Rw = torch.as_tensor(view.R, dtype=F64)
        tw = torch.as_tensor(view.t, dtype=F64)
        p = mu_c @ Rw.T + tw[None, :]
        x, y, z = p[:, 0], p[:, 1], p[:, 2]
        zs = torch.where(z > pp.NEAR_PLANE, z, torch.ones_like(z))
        fx, fy = float(view.fx), float(view.fy)
        zero = torch.zeros_like(zs)
        J = torch.stack([torch.stack([fx / zs, zero, zero], -1),
                         torch.stack([zero, fy / zs, zero], -1)], -2)
        T = J @ Rw
        Sp = T @ S_c @ T.transpose(-1, -2) + pp.DILATION * torch.eye(2, dtype=F64)
        mean2d = torch.stack([fx * x / zs + float(view.cx), fy * y / zs + float(view.cy)], -1)
        return mean2d, Sp, z
    mp.setattr(pp, "project", project)


PY_MUTANTS = {
    "conic_swap_ac": _m_conic_swap_ac,
    "conic_flip_b": _m_conic_flip_b,
    "no_dilation": _m_no_dilation,
    "camera_center_sign": _m_camera_center_sign,
    "query_reversed": _m_query_reversed,
    "query_order_dt": _m_query_order_dt,
    "whitening_transposed": _m_whitening_transposed,
    "opacity_exponent_unscaled": _m_opacity_exponent,
    "beta_map_unscaled": _m_beta_map,
    "beta_tilde_max": _m_beta_tilde_max,
    "condition_mean_sign": _m_condition_mean_sign,
    "condition_cov_unmodulated": _m_condition_cov_unmodulated,
    "condition_not_symmetrised": _m_condition_not_symmetrised,
    "rotation_transposed": _m_rotation_transposed,
    "lqx_transposed": _m_lqx_transposed,
    "jacobian_no_depth_term": _m_jacobian_no_depth_term,
}


def test_unmutated_oracle_passes_every_pin():
    assert _first_failing_pin() is None


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_python_mutant_fails_a_pin(name, monkeypatch):
    PY_MUTANTS[name](monkeypatch)
    assert _first_failing_pin() is not None, f"mutant {name} passes every pin"


# ------------------------------------------------------------------ C mutants
# (original text, mutated text): each original must occur exactly once
C_MUTANTS = {
    "pixel_conic_b_sign": ("double q = r[2] * dx * dx + 2.0 * r[3] * dx * dy + r[4] * dy * dy;",
                           "double q = r[2] * dx * dx - 2.0 * r[3] * dx * dy + r[4] * dy * dy;"),
    "pixel_conic_swap_ac": ("double q = r[2] * dx * dx + 2.0 * r[3] * dx * dy + r[4] * dy * dy;",
                            "double q = r[4] * dx * dx + 2.0 * r[3] * dx * dy + r[2] * dy * dy;"),
    "colour_without_transmittance": ("col[0] += r[8] * alpha * T;", "col[0] += r[8] * alpha;"),
    "kernel_base_sign": ("double base = 1.0 - q;", "double base = 1.0 + q;"),
    "stop_as_skip": ("if (test < T_STOP) break;", "if (test < T_STOP) continue;"),
    "no_alpha_skip": ("if (alpha < ALPHA_MIN) continue;", ""),
    "no_alpha_clamp": ("double alpha = sigma < ALPHA_MAX ? sigma : ALPHA_MAX;", "double alpha = sigma;"),
    "adjoint_ignores_clamp": ("if (c->sigma < ALPHA_MAX) {", "if (1) {"),
    "adjoint_tfinal_sign": ("- gT * Tf / (1.0 - a);", "+ gT * Tf / (1.0 - a);"),
    "adjoint_cross_term": ("t[3] = dq * 2.0 * c->dx * c->dy;", "t[3] = dq * c->dx * c->dy;"),
    "adjoint_behind_colour": ("S[0] = a * r[8] + (1.0 - a) * S[0];", "S[0] = a * r[8] + S[0];"),
    "adjoint_mean_sign": ("t[0] = dq * (-2.0) * (r[2] * c->dx + r[3] * c->dy);",
                          "t[0] = dq * 2.0 * (r[2] * c->dx + r[3] * c->dy);"),
    "tile_edge_minimiser_sign": ("        double t = -(b * dx);\n", "        double t = (b * dx);\n"),
    "tile_margin_dropped": ("double rb = rho * (1.0 + 0x1p-10);", "double rb = rho * (1.0 - 0x1p-6);"),
    "key_without_depth": ("keys[k] = (tile << 32) | (uint64_t)dbits;", "keys[k] = (tile << 32);"),
}


@pytest.fixture(scope="module")
def c_source():
    return open(obuild.SRC).read()


@pytest.mark.parametrize("name", sorted(C_MUTANTS))
def test_c_mutant_fails_a_pin(name, c_source, tmp_path, monkeypatch):
    old, new = C_MUTANTS[name]
    assert c_source.count(old) == 1, f"mutation site of {name} not unique in raster.c"
    src = tmp_path / "raster_mutant.c"
    src.write_text(c_source.replace(old, new))
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                    "-fno-fast-math", "-o", str(lib), str(src), "-lm"], check=True)
    raster.lib()                                  # the oracle's own build exists
    monkeypatch.setattr(raster, "_lib", raster.load(str(lib)))
    assert _first_failing_pin() is not None, f"mutant {name} passes every pin"


def test_mutation_sites_cover_the_record_pipeline():
    """Every record field the compositing reads is touched by some C mutant
    or pinned through a Python mutant of the step that produces it."""
    touched = " ".join(o for o, _ in C_MUTANTS.values())
    for needle in ("r[2]", "r[3]", "r[4]", "r[8]", "T_STOP", "ALPHA_MIN", "ALPHA_MAX", "dbits"):
        assert needle in touched, needle
    assert os.path.exists(obuild.SRC)
    assert np.isfinite(1.0)
