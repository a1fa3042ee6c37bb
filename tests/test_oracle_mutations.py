"""The pins must catch plausible mistakes in the oracle.  Each case plants one
mistake in a copy of the oracle source (a flipped sign, a dropped term, a
swapped operand), builds it on the CPU and checks that the named pins fail
against it.  The real oracle is never modified."""
import os
import subprocess
import sys

import pytest

from oracle import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, original text, mutated text, pins expected to fail)
MUTATIONS = [
    ("ct_corner_sign", "0.25 * (dbm - dbp)", "0.25 * (dbp - dbm)",
     "test_oracle_point.py::test_ct_plane_parallel_reduction"),
    ("ct_upwind_swapped", "if (mflux > 0.0) return lower;", "if (mflux > 0.0) return upper;",
     "test_oracle_point.py::test_ct_upwind_selection"),
    ("minmod_max", "return a < b ? a : b;", "return a < b ? b : a;",
     "test_oracle_point.py::test_plm_brute_force_tiny"),
    ("fast_speed_sign", "s * s - 4.0 * a2 * bn2", "s * s + 4.0 * a2 * bn2",
     "test_oracle_point.py::test_fast_speed_special_cases"),
    ("flux_drops_bn2", "f[1] = rho * vn * vn + pt - bn * bn;", "f[1] = rho * vn * vn + pt;",
     "test_oracle_point.py::test_static_flux test_oracle_point.py::test_hlld_isolated_stationary_contact"),
    ("flux_energy_term", "f[4] = (en + pt) * vn - bn * vb;", "f[4] = (en + pt) * vn;",
     "test_oracle_point.py::test_flux_jacobian_eigenvalues"),
    ("hlld_star_energy_term", "+ pts * sm + bn * (vb - vbs)) / sms;", "+ bn * (vb - vbs)) / sms;",
     "test_oracle_point.py::test_hlld_isolated_stationary_contact "
     "test_oracle_point.py::test_hlld_isolated_rotational_discontinuity"),
    ("hlld_degenerate_star_drops_field", "    bt1s = w[5];\n    bt2s = w[6];\n  } else {",
     "    bt1s = 0.0;\n    bt2s = 0.0;\n  } else {",
     "test_oracle_point.py::test_hlld_degenerate_star_denominator_stationary_contact"),
    ("hll_fallback_ignores_star_pressure",
     "!(star_pressure(&str, sm, bn, gamma) > 0.0))\n      ok = 0;",
     "!(star_pressure(&str, sm, bn, gamma) > 0.0))\n      ok = ok;",
     "test_oracle_point.py::test_hll_fallback_on_negative_star_thermal_pressure"),
    ("hlld_star_velocity_sign", "vt1s = w[2] - bn * w[5] * (sm - w[1]) / dd;",
     "vt1s = w[2] + bn * w[5] * (sm - w[1]) / dd;",
     "test_oracle_scheme.py::test_linear_magnetosonic_waves_second_order"),
    ("hlld_double_star_sign", "(str.bt1 - stl.bt1) * sgn) / (sql + sqr);",
     "(stl.bt1 - str.bt1) * sgn) / (sql + sqr);",
     "test_oracle_point.py::test_hlld_isolated_rotational_discontinuity"),
    ("face_rate_sign", "b->RB[d][c0] = -(t1 - t2);", "b->RB[d][c0] = (t1 - t2);",
     "test_oracle_scheme.py::test_cp_alfven_linear_amplitude"),
    ("bc_wrong_index", "b->Bc[1][c] = 0.5 * (b->B[1][c] + b->B[1][IX(b, i, j + 1, k)]);",
     "b->Bc[1][c] = 0.5 * (b->B[1][c] + b->B[1][IX(b, i + 1, j, k)]);",
     "test_oracle_scheme.py::test_cp_alfven_axes_equivalent"),
    ("rk2_combine", "case 1: return 0.5 * (u0 + (u + dtl));",
     "case 1: return 0.5 * (u0 + u) + dtl;",
     "test_oracle_scheme.py::test_sod_shock_tube_against_exact"),
    ("rk3_second_weights", "case 2: return 0.75 * u0 + 0.25 * (u + dtl);",
     "case 2: return 0.25 * u0 + 0.75 * (u + dtl);",
     "test_oracle_scheme.py::test_rk_temporal_order"),
    ("rk3_third_weights", "default: return (1.0 / 3.0) * u0 + (2.0 / 3.0) * (u + dtl);",
     "default: return 0.5 * u0 + 0.5 * (u + dtl);",
     "test_oracle_scheme.py::test_rk_temporal_order"),
    ("divergence_sign", "r = r - (b->FH[e][m][up[e]] - b->FH[e][m][c]) / b->dx[e];",
     "r = r + (b->FH[e][m][up[e]] - b->FH[e][m][c]) / b->dx[e];",
     "test_oracle_scheme.py::test_sod_shock_tube_against_exact"),
    ("dt_ignores_velocity", "double l = (fabs(w[1 + d]) + cf) / b->dx[d];",
     "double l = cf / b->dx[d];",
     "test_oracle_scheme.py::test_uniform_dt_closed_form"),
    ("periodic_ghost_off_by_one", "while (i < 0) i += n;", "while (i < 0) i += n - 1;",
     "test_oracle_scheme.py::test_conservation_divb_mean_field"),
    ("char_switch_ignored", "  if (rec == ORC_REC_CHAR) {", "  if (0) {",
     "test_oracle_point.py::test_char_slope_limits_each_wave_separately"),
    ("char_left_fast_sign", "L[0][1] = -N * af * cf;", "L[0][1] = N * af * cf;",
     "test_oracle_point.py::test_prim_eigenvectors_solve_the_jacobian"),
    ("char_alfven_field_sign", "R[5][1] = -sg * sr * bez;", "R[5][1] = sg * sr * bez;",
     "test_oracle_point.py::test_prim_eigenvectors_solve_the_jacobian"),
    ("char_alpha_slow", "double as2 = 0.5 * (sm + bt2) / sq;", "double as2 = 0.5 * (sm - bt2) / sq;",
     "test_oracle_point.py::test_prim_eigenvectors_solve_the_jacobian"),
    ("emf_e0_upwinds", "if (kind == ORC_EMF_E0) return orc_ct_corner(fa1, fa0, fb1, fb0, ec, 0.0, 0.0, 0.0, 0.0);",
     "if (kind == ORC_EMF_E0) return orc_ct_corner(fa1, fa0, fb1, fb0, ec, ma1, ma0, mb1, mb0);",
     "test_oracle_point.py::test_ct_corner_kinds"),
    ("emf_arith_drops_face", "if (kind == ORC_EMF_ARITH) return 0.25 * (fa1 + fa0 + fb1 + fb0);",
     "if (kind == ORC_EMF_ARITH) return 0.25 * (fa1 + fa0 + fb1 + fb1);",
     "test_oracle_point.py::test_ct_corner_kinds"),
    ("mc_bound_one_sided", "double m = 2.0 * a < 2.0 * b ? 2.0 * a : 2.0 * b;",
     "double m = 2.0 * a < 2.0 * b ? a : b;",
     "test_oracle_point.py::test_limiters_match_their_flux_limiter_functions"),
    ("vanleer_arithmetic_mean", "return 2.0 * a * b / (a + b);", "return 0.5 * (a + b);",
     "test_oracle_point.py::test_limiters_match_their_flux_limiter_functions"),
    ("limiter_switch_ignored", "if (b->rec == ORC_REC_PRIM && b->lim == ORC_LIM_MINMOD) {",
     "if (b->rec == ORC_REC_PRIM) {",
     "test_oracle_scheme.py::test_limiters_sod_order_and_sharpness"),
    ("hll_switch_ignored", "if (b->solver == ORC_HLL) {", "if (0) {",
     "test_oracle_scheme.py::test_hll_stationary_contact_closed_form"),
    ("hll_upwind_term_sign", "f[c] = (sr * fL[c] - sl * fR[c] + sl * sr * (uR[c] - uL[c])) / (sr - sl);",
     "f[c] = (sr * fL[c] - sl * fR[c] - sl * sr * (uR[c] - uL[c])) / (sr - sl);",
     "test_oracle_scheme.py::test_hll_stationary_contact_closed_form"),
    ("uct_diffusion_sign", "return num / (sa * sb) - apb * amb / sb * (ba[1] - ba[0]) +",
     "return num / (sa * sb) + apb * amb / sb * (ba[1] - ba[0]) +",
     "test_oracle_point.py::test_uct_hll_reduces_to_hll_along_each_axis "
     "test_oracle_scheme.py::test_uct_hll_1d_equals_the_hll_face_flux"),
    ("uct_weights_swapped", "double num = apa * apb * e[0] + ama * apb * e[1]",
     "double num = ama * apb * e[0] + apa * apb * e[1]",
     "test_oracle_point.py::test_uct_hll_upwind_uniform_and_mirror"),
    ("uct_corner_slope_side", "return side == 0 ? q0 + 0.5 * d : q0 - 0.5 * d;",
     "return side == 0 ? q0 - 0.5 * d : q0 + 0.5 * d;",
     "test_oracle_scheme.py::test_uct_hll_1d_equals_the_hll_face_flux"),
    ("uct_speed_bound_from_left_speed",
     "alpha[2 * e] = speed_bound(b->SP[d][1][i0], b->SP[d][1][i1], 0);",
     "alpha[2 * e] = speed_bound(b->SP[d][0][i0], b->SP[d][0][i1], 0);",
     "test_oracle_scheme.py::test_uct_hll_1d_equals_the_hll_face_flux"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,orig,mut,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, orig, mut, pins):
    src = open(B.SRC).read()
    assert src.count(orig) >= 1, f"mutation anchor for {name} not found"
    mutated = src.replace(orig, mut, 1)
    msrc = tmp_path / "mutant.c"
    msrc.write_text(mutated)
    lib = B.compile_to(str(msrc), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, MHD_ORACLE_LIB=lib)
    args = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"]
    args += [os.path.join(ROOT, "tests", p) for p in pins.split()]
    r = subprocess.run(args, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins {pins} did not catch mutation {name}:\n{r.stdout[-2000:]}"
