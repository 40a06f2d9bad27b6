"""Planted mistakes: each copy of the oracle with one plausible error must
fail at least one pin.  The mistakes are planted in a temporary copy of the
oracle source, compiled with the oracle's own recipe, on the CPU."""
import os

import pytest

import oracle as O
import oracle_checks as C

MUTATIONS = [
    # (name, text in the oracle source, planted replacement, pins expected to catch it)
    ("equilibrium_printed_coefficient", "uu_cc / (2.0 * CS2 * CS2)", "uu_cc / (2.0 * CS2)",
     [C.check_equilibrium_moments, C.check_moments_round_trip]),
    ("pressure_drops_rho0_term", "(1.0 - OMEGA[0]) * rho0", "(1.0 - OMEGA[0]) * 0.0",
     [C.check_moments_round_trip]),
    ("upwind_printed_third_point", "at(p, plane, i + 2 * di, j + 2 * dj)", "at(p, plane, i + di, j + dj)",
     [C.check_stencils_on_quartics]),
    ("upwind_side_inverted", "    if (ORC_UPWIND_NONNEG(c)) {", "    if (!ORC_UPWIND_NONNEG(c)) {",
     [C.check_stencils_on_quartics]),
    ("one_sided_fallback_wrong", "upwind = (c0 - m1) / h;", "upwind = (c0 - m1) / (2.0 * h);",
     [C.check_metric_exact_on_linear_fields]),
    ("metric_xi_y_sign", "xi_y = -x_eta / jac", "xi_y = x_eta / jac",
     [C.check_metric_exact_on_linear_fields]),
    ("jacobian_missing", "orc_real xi_x = y_eta / jac", "orc_real xi_x = y_eta",
     [C.check_metric_exact_on_linear_fields]),
    ("map_sign", "*x = 2.0 * C * xi * eta + xi - C * eta + C;", "*x = 2.0 * C * xi * eta + xi + C * eta + C;",
     [C.check_geometry_matches_paper]),
    ("shear_rate_missing_factor_two", "orc_real gamma2 = 2.0 * (Dxx", "orc_real gamma2 = 1.0 * (Dxx",
     [C.check_relaxation_time_power_law, C.check_couette_power_law]),
    ("strain_uses_lambda_twice", "-sxx / (lam_old * CS2)", "-sxx / (2.0 * lam_old * CS2)",
     [C.check_relaxation_time_power_law, C.check_couette_power_law]),
    ("fbar_plus_coefficient", "3.0 * dt / (4.0 * lam + 2.0 * dt) * feq[k]", "2.0 * dt / (4.0 * lam + 2.0 * dt) * feq[k]",
     [C.check_conversions_follow_definitions, C.check_collision_invariants, C.check_exact_conservation_periodic]),
    ("fhat_from_f_coefficient", "f[k] = 2.0 * lam / (2.0 * lam + dt) * fh[k]", "f[k] = lam / (2.0 * lam + dt) * fh[k]",
     [C.check_conversions_follow_definitions]),
    ("fbar_to_f_coefficient", "f[k] = 4.0 * lam / (4.0 * lam + dt) * fb[k]", "f[k] = 2.0 * lam / (4.0 * lam + dt) * fb[k]",
     [C.check_conversions_follow_definitions]),
    ("half_step_full_dt", "- 0.5 * dt * stream_term(p, d, w->fbar_plus", "- 1.0 * dt * stream_term(p, d, w->fbar_plus",
     [C.check_taylor_green_decay]),
    ("nee_uses_fluid_velocity", "orc_equilibrium(P, wx, wy, p->rho0, feq_w);", "orc_equilibrium(P, ux, uy, p->rho0, feq_w);",
     [C.check_couette_power_law]),
    ("lattice_diagonals_swapped", "static const double CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};",
     "static const double CX[9] = {0, 1, 0, -1, 0, -1, 1, -1, 1};",
     [C.check_lattice_matches_paper]),
    ("energy_edge_weights", "? 0.5 : 1.0;\n            orc_real wj", "? 1.0 : 1.0;\n            orc_real wj",
     [C.check_kinetic_energy_weights]),
    ("implicit_strain_scale", "orc_real s = 2.0 * lam + dt;", "orc_real s = lam + dt;",
     [C.check_implicit_lambda]),
    ("implicit_bracket_direction", "            lo = mid;\n        else", "            hi = mid;\n        else",
     [C.check_implicit_lambda]),
    ("viscosity_from_consistency", "return mu / CS2;", "return mu * CS2;",
     [C.check_relaxation_time_power_law, C.check_taylor_green_decay]),
    ("initial_lambda_drops_cs2", "d->lam0 = U / (p->re * CS2);", "d->lam0 = U / p->re;",
     [C.check_initial_lambda]),
    ("initial_lambda_newtonian_only", "d->lam0 = U / (p->re * CS2);", "d->lam0 = pow(U, 2.0 - p->n) / (p->re * CS2);",
     [C.check_initial_lambda]),
]


@pytest.mark.parametrize("name,find,plant,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(tmp_path, name, find, plant, pins):
    src = open(os.path.join(os.path.dirname(O.__file__), "ifdlbm_oracle.c")).read()
    assert src.count(find) == 1, "the text to mutate must occur exactly once: %r" % find
    path = tmp_path / ("oracle_%s.c" % name)
    path.write_text(src.replace(find, plant))
    lib = O.compile_source(str(path), str(tmp_path / ("liboracle_%s.so" % name)))
    caught = []
    with O.using(lib):
        for pin in pins:
            try:
                pin()
            except (AssertionError, FloatingPointError, ValueError, ZeroDivisionError, OverflowError):
                caught.append(pin.__name__)
    assert caught, "no pin caught the planted mistake %s" % name
