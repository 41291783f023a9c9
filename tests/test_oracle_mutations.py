"""Plant plausible mistakes in a copy of the C oracle and show that the pins
catch each of them.  Runs entirely on the CPU; the real oracle is untouched."""
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_forward_euler as fe
from tests import test_oracle_mds_fnode as mf
from tests import test_oracle_paper_models as pm
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, exact text in oracle.c, replacement, pins expected to catch it)
MUTATIONS = [
    ("vdp_jacobian_sign", "J[2] = -2.0 * mu * y[0] * y[1] - 1.0;", "J[2] = 2.0 * mu * y[0] * y[1] - 1.0;",
     [lambda: pins.test_model_jacobian_matches_central_differences(pins._model_cases()[1])]),
    ("robertson_dropped_term", "f[1] = k1 * y[0] - k3 * y[1] * y[2] - k2 * y[1] * y[1];",
     "f[1] = k1 * y[0] - k3 * y[1] * y[2];",
     [pins.test_robertson_mass_conservation, pins.test_robertson_first_order_convergence]),
    ("newton_dt_sign", "J[i * n + c] = (i == c ? 1.0 : 0.0) - dt * J[i * n + c];",
     "J[i * n + c] = (i == c ? 1.0 : 0.0) + dt * J[i * n + c];",
     [pins.test_lin_exact_be_recurrence]),
    ("adjoint_untransposed", "Dt[c * n + i] = (i == c ? 1.0 : 0.0) - dt * J[i * n + c];",
     "Dt[i * n + c] = (i == c ? 1.0 : 0.0) - dt * J[i * n + c];",
     [pins.test_lin_adjoint_closed_form, pins.test_adjoint_fd_vanderpol]),
    ("adjoint_dropped_g0", "pb->dLdy0[b * n + i] = G[i] + lam[i];", "pb->dLdy0[b * n + i] = lam[i];",
     [pins.test_lin_adjoint_closed_form]),
    ("mlp_vjp_dropped_tanh_derivative",
     "for (int i = 0; i < H; ++i) s += W2[i * H + k] * d2[i];\n            d1[k] = s * (1.0 - a1[k] * a1[k]);",
     "for (int i = 0; i < H; ++i) s += W2[i * H + k] * d2[i];\n            d1[k] = s;",
     [lambda: pins.test_model_param_vjp_matches_central_differences(pins._model_cases()[3])]),
    ("mlp_w2_transposed", "for (int k = 0; k < H; ++k) s += W2[i * H + k] * a1[k];",
     "for (int k = 0; k < H; ++k) s += W2[k * H + i] * a1[k];",
     [pins.test_model_rates_match_independent_definitions]),
    ("lu_wrong_pivot", "if (v > best) { best = v; piv = r; }", "if (v < best) { best = v; piv = r; }",
     [pins.test_lu_matches_numpy_and_pivots]),
    ("vdp_param_vjp_wrong_component", "gp[0] += w[1] * (1.0 - y[0] * y[0]) * y[1];",
     "gp[0] += w[0] * (1.0 - y[0] * y[0]) * y[1];",
     [lambda: pins.test_model_param_vjp_matches_central_differences(pins._model_cases()[1])]),
    ("fe_update_sign", "Y[k * n + i] = yp[i] + dt * f[i];", "Y[k * n + i] = yp[i] - dt * f[i];",
     [fe.test_fe_linear_closed_form, fe.test_fe_vdp_mu_zero_is_a_growing_rotation]),
    ("fe_rate_at_wrong_time_point", "rhs(kind, n, H, yp, t[k - 1], p, f, NULL);",
     "rhs(kind, n, H, yp + (k > 1 ? -n : 0), t[k - 1], p, f, NULL);",
     [fe.test_fe_linear_closed_form]),
    ("fe_adjoint_untransposed", "s += dt1 * J[r * n + i] * lam[r];", "s += dt1 * J[i * n + r] * lam[r];",
     [fe.test_fe_adjoint_linear_closed_form, fe.test_fe_adjoint_fd_vanderpol]),
    ("fe_adjoint_param_term_at_new_state", "vjp_p(kind, n, H, Y + (k - 1) * n, t[k - 1], p, w, gp);",
     "vjp_p(kind, n, H, Y + k * n, t[k - 1], p, w, gp);",
     [fe.test_fe_adjoint_linear_closed_form, fe.test_fe_adjoint_fd_vanderpol]),
    ("chaboche_hardening_without_plastic_rate", "f[1] = tau * (Kinf - y[1]) * c.pa;",
     "f[1] = tau * (Kinf - y[1]);",
     [lambda: pm.test_rate_jacobian_and_parameter_gradient_match_autograd(pm._cases()[3])]),
    ("chaboche_jacobian_sign", "dep[1] = -c.dpa * c.sg;", "dep[1] = c.dpa * c.sg;",
     [lambda: pm.test_rate_jacobian_and_parameter_gradient_match_autograd(pm._cases()[0])]),
    ("neuron_vjp_sign", "g[NR_TM] -= w[4 * i + 1] * (q[NR_MINF] - m) / (q[NR_TM] * q[NR_TM]);",
     "g[NR_TM] += w[4 * i + 1] * (q[NR_MINF] - m) / (q[NR_TM] * q[NR_TM]);",
     [lambda: pm.test_rate_jacobian_and_parameter_gradient_match_autograd(pm._cases()[9])]),
    ("neuron_coupling_jacobian", "r[4 * j] = (j == i) ? 0.0 : -q[NR_GC] / q[NR_C];",
     "r[4 * j] = (j == i) ? 0.0 : q[NR_GC] / q[NR_C];",
     [lambda: pm.test_rate_jacobian_and_parameter_gradient_match_autograd(pm._cases()[10])]),
    # mass-damper-spring: a damper acting one unit off, a spring dividing by the
    # neighbour's mass, the wall not holding, the force on the wrong mass
    ("mds_damper_index", "if (i > 0) a -= K[i - 1] * (d - y[2 * i - 2]) + C[i - 1] * (v - y[2 * i - 1]);",
     "if (i > 0) a -= K[i - 1] * (d - y[2 * i - 2]) + C[i] * (v - y[2 * i - 1]);",
     [lambda: mf.test_mds_momentum_balance_every_step(2), lambda: mf.test_mds_backward_euler_energy_identity(2, True),
      lambda: mf.test_mds_rate_and_jacobian_match_element_assembly(2)]),
    ("mds_spring_over_neighbour_mass", "*acc = a / M[i];", "*acc = a / M[i + 1 < nu ? i + 1 : i];",
     [lambda: mf.test_mds_momentum_balance_every_step(2), lambda: mf.test_mds_backward_euler_energy_identity(2, False)]),
    ("mds_wall_released", "const double dn = (i + 1 < nu) ? y[2 * i + 2] : 0.0, vn = (i + 1 < nu) ? y[2 * i + 3] : 0.0;\n    double a",
     "const double dn = (i + 1 < nu) ? y[2 * i + 2] : y[2 * i], vn = (i + 1 < nu) ? y[2 * i + 3] : y[2 * i + 1];\n    double a",
     [lambda: mf.test_mds_momentum_balance_every_step(1), mf.test_mds_single_unit_converges_to_forced_oscillator]),
    ("mds_force_sign", "f[2 * i + 1] = a + (i == 0 ? p[3 * nu] * sin(", "f[2 * i + 1] = a - (i == 0 ? p[3 * nu] * sin(",
     [lambda: mf.test_mds_momentum_balance_every_step(2), mf.test_mds_single_unit_converges_to_forced_oscillator]),
    # forced neural ODE: the output tanh dropped, the forcing fed at the wrong input
    ("fnode_output_tanh_dropped", "J[i * n + c] = (1.0 - f[i] * f[i]) * s;", "J[i * n + c] = s;",
     [lambda: mf.test_fnode_rate_jacobian_and_parameter_gradient_match_autograd(5)]),
    ("fnode_forcing_input_column", "gx += q.W1[i * m + n] * d1[i];", "gx += q.W1[i * m] * d1[i];",
     [lambda: mf.test_fnode_rate_jacobian_and_parameter_gradient_match_autograd(5)]),
]


@pytest.mark.parametrize("mut", MUTATIONS, ids=lambda m: m[0])
def test_pins_catch_planted_mistake(mut, tmp_path):
    name, old, new, checks = mut
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found exactly once: " + name
    path = tmp_path / "oracle.c"
    path.write_text(src.replace(old, new))
    (tmp_path / "oracle.h").write_text(open(SRC[:-2] + ".h").read())
    lib = tmp_path / ("liboracle_%s.so" % name)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", str(lib), str(path),
                           "-lm", "-lpthread"])
    caught = 0
    with oracle.using_library(str(lib)):
        for check in checks:
            try:
                check()
            except Exception:  # an assertion or a failure status the pin turns into an error
                caught += 1
    assert caught == len(checks), "%s: only %d of %d pins caught it" % (name, caught, len(checks))
