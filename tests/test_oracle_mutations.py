"""The oracle's pins catch plausible mistakes.

Each case plants one mistake (a dropped term, a wrong sign, a wrong power or
coefficient) in a private copy of the oracle's C source, builds that copy on
the CPU, and runs the pin that should reject it.  The real oracle is never
touched.
"""
import importlib.util
import os
import shutil
import sys

import pytest

import tests.test_oracle_adjoint as T_adj
import tests.test_oracle_force as T_force
import tests.test_oracle_integrator as T_int

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                          "oracle")

MUTATIONS = [
    # (id, text in nbody_oracle.c, replacement, pin that must fail)
    ("sign_of_separation", "rx = pos[j] - xi;", "rx = xi - pos[j];",
     lambda o: T_force.test_circular_binary_closed_form(o, 0.05)),
    ("jerk_coefficient", "jx += mj * (vx * r3inv - 3.0 * rv", "jx += mj * (vx * r3inv - 2.0 * rv",
     T_force.test_jerk_is_time_derivative_of_acceleration),
    ("jerk_power", "r5inv = r3inv * rinv * rinv;      /* s^(-5/2) */", "r5inv = r3inv * rinv;",
     T_force.test_jerk_is_time_derivative_of_acceleration),
    ("softening_placement", "s2 = rx * rx + ry * ry + rz * rz + eps2;",
     "s2 = rx * rx + ry * ry + rz * rz + 2.0 * eps2;",
     lambda o: T_force.test_circular_binary_closed_form(o, 0.3)),
    ("potential_power", "ph -= mj * rinv;", "ph -= mj * rinv * rinv;",
     T_force.test_acceleration_is_minus_gradient_of_potential),
    ("dropped_y_velocity", "vy = vel[n_j + j] - vi;", "vy = vel[n_j + j];",
     T_force.test_jerk_is_time_derivative_of_acceleration),
    ("predictor_coefficient", "(dt / 3.0) * k[q]", "(dt / 2.0) * k[q]",
     T_int.test_predictor_exact_on_cubics),
    ("corrector_x_coefficient", "(A2 / 12.0 + A3 / 20.0)", "(A2 / 6.0 + A3 / 20.0)",
     T_int.test_corrector_exact_on_quintics),
    ("corrector_a3_sign", "2.0 * (a0 - a1) + (k0 + k1) * h", "2.0 * (a0 - a1) + (k0 - k1) * h",
     T_int.test_corrector_exact_on_quintics),
    ("corrector_v_term", "(A2 / 3.0 + A3 / 4.0) * h", "(A2 / 3.0) * h",
     T_int.test_corrector_exact_on_quintics),
    ("criterion_jerk_square", "eta * (an * a2n + kn * kn)", "eta * (an * a2n + kn)",
     lambda o: T_int.test_aarseth_step_closed_form_on_circular_orbit(o, 1.15, -6, 0.0, -6)),
    ("criterion_a2_end_of_step", "(2.0 * A2 + 6.0 * A3) / (h * h)", "(2.0 * A2) / (h * h)",
     T_int.test_step_criterion_uses_end_of_step_derivatives),
    ("doubling_ignores_commensurability", "fmod(t_new, 2.0 * d) == 0.0 &&", "",
     lambda o: T_int.test_aarseth_step_closed_form_on_circular_orbit(o, 2.15, -6, 0.0, -6)),
    ("energy_half_factor", "out[1] = 0.5 * wsum;", "out[1] = wsum;",
     T_int.test_two_body_energy_closed_form),
    ("adjoint_third_order_term", "15.0 * q * ga * kr", "5.0 * q * ga * kr",
     lambda o: T_adj.test_dot_product_identity(o, 0.05)),
    ("adjoint_velocity_term", "gv[c] = mj * (al * K[c] - 3.0 * be * kr * r[c]);",
     "gv[c] = mj * (al * K[c]);",
     lambda o: T_adj.test_dot_product_identity(o, 0.0)),
    ("initial_step_ignores_nonfinite_norms", "!(want == want) || !isfinite(an) || !isfinite(kn)",
     "!(want == want)", T_int.test_initial_step_flags_nonfinite_norms),
    ("corrector_ignores_nonfinite_state", "if (bad) rc = ORC_E_NONFINITE;", "",
     lambda o: T_int.test_corrector_reports_nonfinite_state(o, True)),
    ("sorted_largest_first", "if (a->key < b->key) return -1;", "if (a->key > b->key) return -1;",
     T_force.test_sorted_sum32_keeps_small_forces_that_index_order_drops),
    ("sum32_in_float64", "float sum[7] = {", "double sum[7] = {",
     T_force.test_sorted_sum32_keeps_small_forces_that_index_order_drops),
    ("sorted_key_ignores_mass", "keys[m].key = fabs(mj) * sqrt", "keys[m].key = sqrt",
     T_force.test_sorted_sum32_orders_by_force_not_distance),
]


def _mutant(tmp_path, name, old, new):
    d = tmp_path / ("oracle_" + name)
    shutil.copytree(ORACLE_DIR, d, ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    src = d / "nbody_oracle.c"
    text = src.read_text()
    assert text.count(old) >= 1, "mutation anchor not found: " + old
    src.write_text(text.replace(old, new, 1))
    modname = "oracle_mutant_" + name
    spec = importlib.util.spec_from_file_location(modname, str(d / "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    sys.modules[modname] = mod
    spec.loader.exec_module(mod)
    mod.build(force=True)
    return mod


@pytest.mark.parametrize("name,old,new,pin", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_rejects_planted_mistake(tmp_path, orc, name, old, new, pin):
    pin(orc)  # the real oracle passes the pin
    mut = _mutant(tmp_path, name, old, new)
    with pytest.raises(AssertionError):
        pin(mut)
