"""The pins catch plausible mistakes: each case plants one in a private copy of
the oracle's C source (never in the committed oracle), builds it, and checks
that at least one pin fails against the mutated build."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import test_oracle_pins as pins
from tests import test_oracle_user as upins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, [(old, new), ...]) -- every `old` must occur in the source
MUTATIONS = [
    ("stage4_uses_half_step", [("or_axpy(L, z, dt, k3, tmp)", "or_axpy(L, z, h2, k3, tmp)"),
                               ("tmp[i] = z[i] + dt * k3[i]", "tmp[i] = z[i] + h2 * k3[i]")]),
    ("update_missing_h", [("z[i] = z[i] + h6 * (", "z[i] = z[i] + (1.0 / 6.0) * (")]),
    ("k3_weight_one", [("2.0 * k3[i]", "1.0 * k3[i]")]),
    ("ctm_supply_reads_own_cell", [("? y[i + 1] : 0.0;", "? y[i] : 0.0;")]),
    ("ctm_outflow_has_supply", [("return or_min2(v * yi, q);", "return or_min3(v * yi, w * c, q);")]),
    ("ctm_inflow_nonzero", [("if (g < 0) return 0.0;", "if (g < 0) return q;")]),
    ("lin3_sign_split_swapped", [("or_pos(aL) * xm + or_neg(aL) * hm",
                                  "or_neg(aL) * xm + or_pos(aL) * hm")]),
    ("lin3_input_sides_swapped", [("or_pos(b) * or_input(S, p, i) + or_neg(b) * or_input(S, ph, i)",
                                   "or_pos(b) * or_input(S, ph, i) + or_neg(b) * or_input(S, p, i)")]),
    ("rd_cubic_dropped", [("lap - yi * yi * yi", "lap - yi * yi")]),
    ("rd_diffusion_sign", [("(ym - 2.0 * yi + yp)", "(ym + 2.0 * yi + yp)")]),
    ("rd_spacing_not_squared", [("/ (h * h)", "/ h")]),
    ("mc_wrong_stream", [("#define OR_MC_STREAM 2", "#define OR_MC_STREAM 1")]),
    ("mc_uniform_bits", [("ldexp((double)(w >> 11), -53)", "ldexp((double)(w >> 12), -52)")]),
    ("gb_signed_offdiagonal", [("C[0] = fabs(prm[0]);", "C[0] = prm[0];")]),
    ("gb_center_input_is_lower", [("pc[i] = n_in > 0 ? (p_lo[i] + p_hi[i]) / 2.0 : 0.0;",
                                   "pc[i] = n_in > 0 ? p_lo[i] : 0.0;")]),
    ("gb_radius_not_halved", [("r[i] = (x_hi[i] - x_lo[i]) / 2.0;", "r[i] = (x_hi[i] - x_lo[i]);")]),
    ("gb_ctm_diagonal_negative", [("C[0] = prm[0]; C[1] = 0.0; C[2] = prm[1]; C[3] = 0.0;",
                                   "C[0] = prm[0]; C[1] = -prm[0]; C[2] = prm[1]; C[3] = 0.0;")]),
    ("heat_open_face_insulated", [("if (d == 0 && s == 1) sum += 0.0 - u;",
                                   "if (d == 9 && s == 1) sum += 0.0 - u;")]),
    ("heat_open_face_at_x0", [("if (d == 0 && s == 1) sum += 0.0 - u;",
                               "if (d == 0 && s == -1) sum += 0.0 - u;")]),
    ("heat_all_faces_open", [("continue;                                /* insulated face */",
                              "sum += 0.0 - u; continue;")]),
    ("heat_z_axis_dropped", [("for (d = 0; d < 3; ++d) {\n        for (s = -1;",
                              "for (d = 0; d < 2; ++d) {\n        for (s = -1;")]),
    ("heat_spacing_not_squared", [("alpha / (dx * dx) * sum", "alpha / dx * sum")]),
    ("heat_axes_transposed", [("{i % wx, (i / wx) % wy, i / (wx * wy)}",
                               "{i % wy, (i / wy) % wx, i / (wx * wy)}")]),
    ("user_neighbour_sides_swapped", [("S->user(xm, x[i], xp, hm, xh[i], hp,",
                                       "S->user(hm, x[i], hp, xm, xh[i], xp,")]),
    ("user_inputs_swapped", [("or_input(S, p, i), or_input(S, ph, i),\n                       S->prm",
                              "or_input(S, ph, i), or_input(S, p, i),\n                       S->prm")]),
    ("user_window_index_local", [("(long long)(S->g0 + i), (long long)S->n_total",
                                  "(long long)i, (long long)S->n_total")]),
]

PINS = [
    lambda: pins.test_lin3_trajectory_exact_rational(3, (0.5, -1.25, 0.75, 2.0)),
    lambda: pins.test_lin3_trajectory_exact_rational(4, (-0.375, -0.5, 1.5, -1.0)),
    lambda: pins.test_lin3_embedding_exact_rational(3),
    pins.test_lin3_per_cell_inputs_exact_rational,
    pins.test_rd_dirichlet_sine_mode_decays_by_stability_polynomial,
    pins.test_rd_spacing_scales_diffusion,
    pins.test_rd_single_cell_bernoulli_fourth_order,
    pins.test_ctm_free_flow_regime_exact_rational,
    pins.test_ctm_congested_regime_exact_rational,
    pins.test_ctm_capacity_regime,
    pins.test_ctm_flux_uses_downstream_supply,
    pins.test_uniform_draw_layout,
    pins.test_mc_zero_steps_returns_extreme_draws,
    pins.test_growth_bound_radius_exact_rational,
    pins.test_growth_bound_equals_embedding_on_cooperative_linear_chain,
    lambda: pins.test_contraction_matrix_bounds_the_jacobian(pins.oracle.CTM),
    lambda: pins.test_contraction_matrix_bounds_the_jacobian(pins.oracle.RD),
    lambda: pins.test_heat3d_trajectory_exact_rational((3, 2, 2)),
    lambda: pins.test_heat3d_cosine_mode_decays_by_stability_polynomial((1, 2, 1)),
    pins.test_heat3d_heat_leaves_only_through_the_open_face,
    lambda: upins.test_user_lin3_equals_builtin_bitwise(_users(), (-0.5, -1.0, 0.75, -1.5),
                                                        "cell"),
    lambda: upins.test_user_ctm_equals_builtin_bitwise_whole_and_window(_users()),
]


def _users():
    from tests import user_sources as us
    return {k: oracle.UserSystem(getattr(us, k)) for k in ("LIN3", "CTM")}


def _build_mutant(tmp_path, edits):
    src = open(SRC).read()
    for old, new in edits:
        assert old in src, f"mutation anchor not found: {old!r}"
        src = src.replace(old, new)
    c = tmp_path / "mutant.c"
    so = tmp_path / "libmutant.so"
    c.write_text(src)
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-std=gnu99", str(c), "-o", str(so), "-lm"])
    return str(so)


@pytest.mark.parametrize("name,edits", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, monkeypatch, name, edits):
    so = _build_mutant(tmp_path, edits)
    saved = oracle._lib
    oracle._lib = None
    monkeypatch.setattr(oracle, "_SO", so)
    try:
        oracle.lib()
        caught = []
        for pin in PINS:
            try:
                pin()
            except AssertionError:
                caught.append(pin)
        assert caught, f"no pin caught mutation {name}"
    finally:
        oracle._lib = saved
