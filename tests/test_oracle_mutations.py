"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake (a dropped term, a wrong sign or factor) in a
private copy of the oracle source, builds it, and runs the pin that should
catch it against the mutant in a child pytest; the child must fail.  The
mutants are built and run side by side (a module fixture); this runs on the
CPU only."""
import concurrent.futures
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dlb_oracle.c")

T = "tests/test_oracle_dynamics.py::"
TT = "tests/test_oracle_tables.py::"
TR = "tests/test_oracle_restart.py::"
TS = "tests/test_oracle_stencil.py::"
TH = "tests/test_oracle_heat_substeps.py::"
TF = "tests/test_oracle_farfield.py::"
TFO = "tests/test_oracle_force.py::"
TC = "tests/test_oracle_coupling_pins.py::"
# the anti-trapping current of Sec. 2 as the oracle writes it
JAT = ("double c = -1.0 / (2.0 * sqrt(2.0)) * p->W0 * (1.0 + (1.0 - p->k) * U) * dphi / gnorm;")

MUTATIONS = [
    ("force: K pressure term dropped", "double K = 2.0 * (s2 - 3.0 * s4 + s2 * s4) / (9.0 * s2 * s4);",
     "double K = 0.0;", TFO + "test_forced_porous_medium_is_steady"),
    ("force: u* without F/2", "ustar[0] = mx + 0.5 * F[0];", "ustar[0] = mx;",
     TFO + "test_forced_porous_medium_is_steady"),
    ("force: not rescaled to sub-steps", "F[0] = p->force_x / (n * n);", "F[0] = p->force_x / n;",
     TFO + "test_liquid_accelerates_by_the_force"),
    ("force: sign of the varphi isotropic part", "(2.0 * cu * cF - 2.0 * cs2 * uF)",
     "(2.0 * cu * cF + 2.0 * cs2 * uF)", TFO + "test_forcing_populations_match_the_printed_moments"),
    ("far field: the wall copies its neighbour", "for (int i = 0; i < 5; ++i) d[i] = eb[i] - ef[i];",
     "for (int i = 0; i < 5; ++i) d[i] = 0.0;", TF + "test_relaxes_to_the_far_field_zero_gradient_walls_do_not"),
    ("far field: sign of the equilibrium shift", "for (int i = 0; i < 5; ++i) d[i] = eb[i] - ef[i];",
     "for (int i = 0; i < 5; ++i) d[i] = ef[i] - eb[i];", TF + "test_dirichlet_mode_decays_at_the_diffusion_rate"),
    ("far field: C of U0 without the 1 - k factor",
     "* (1.0 + (1.0 - p->k) * p->U0) : p->C0;", "* (1.0 + p->U0) : p->C0;",
     TF + "test_relaxes_to_the_far_field_zero_gradient_walls_do_not"),
    ("heat sub-steps: velocity in main-step units", "s->ux[x] / ns, s->uy[x] / ns, geq", "s->ux[x], s->uy[x], geq",
     TH + "test_advected_heat_mode_with_sub_steps"),
    ("heat sub-steps: diffusivity not rescaled", "1.0 / (3.0 * p->alpha / heat_sub(p) + 0.5)",
     "1.0 / (3.0 * p->alpha + 0.5)", TH + "test_heat_mode_decays_at_alpha_per_main_step"),
    ("heat sub-steps: d_t(Hu) in main-step units", "(s->Hu[x] - s->Hu_prev[x]) / ((double)ns * ns)",
     "(s->Hu[x] - s->Hu_prev[x]) / (double)ns", TH + "test_advected_heat_mode_with_sub_steps"),
    ("stencil gradient: sign of the y part", "gy += 3.0 * W9[i] * C9Y[i] * F[yy * nx + xx];",
     "gy -= 3.0 * W9[i] * C9Y[i] * F[yy * nx + xx];", TS + "test_stencil_is_exact_on_quadratics"),
    ("stencil gradient: 1/cs^2 taken as 2", "gx += 3.0 * W9[i] * C9X[i] * F[yy * nx + xx];",
     "gx += 2.0 * W9[i] * C9X[i] * F[yy * nx + xx];", TS + "test_stencil_is_exact_on_quadratics"),
    ("stencil mode without anisotropy", "aniso_or_hook(p, lg[0], lg[1], &lg[2], &lg[3], &lg[4]);",
     "lg[2] = 1.0, lg[3] = lg[4] = 0.0;", TS + "test_planar_front_is_stationary_with_the_stencil_gradient"),
    ("no d_t F^phi term (Remark 2)", "acc += F[i] + 0.5 * a2 * dF[i];", "acc += F[i];",
     T + "test_phase_field_mode_decay_with_fixed_anisotropy"),
    ("plain streaming for phi", "(s->pf[o + src] - s->f[o + d]) / s->a2[src]",
     "(s->pf[o + src] - s->f[o + d])", T + "test_phase_field_mode_decay_with_fixed_anisotropy"),
    ("sign of G^phi", "G[i] = -W5[i] * (C5X[i] * Nx + C5Y[i] * Ny) / a2;",
     "G[i] = W5[i] * (C5X[i] * Nx + C5Y[i] * Ny) / a2;",
     T + "test_front_undulation_relaxes_with_anisotropic_stiffness"),
    ("no d_t(Cu), d_t(Hu)", "double Vx = 3.0 * dCu[0]", "double Vx = 0.0 * dCu[0]",
     T + "test_advected_mode_keeps_the_diffusivity"),
    ("sign of U grad q", "double Vx = 3.0 * dCu[0] + U * (-0.5 * gx)",
     "double Vx = 3.0 * dCu[0] + U * (0.5 * gx)",
     T + "test_uniform_U_and_theta_are_steady_across_a_still_front"),
    ("half the interface force", "Fb[0] = (1.0 - qt) * fx;", "Fb[0] = 0.5 * (1.0 - qt) * fx;",
     TT + "test_fully_solid_node_stops_the_flow"),
    ("phase-field rate without a_s^2", "return 1.0 / (as * as * W2t * 3.0 + 0.5);", "return 1.0 / (W2t * 3.0 + 0.5);",
     T + "test_phase_field_mode_decay_with_fixed_anisotropy"),
    ("solute rate without 1 - k", "double s1c = 1.0 / (3.0 * p->D * (1.0 - p->k) + 0.5);",
     "double s1c = 1.0 / (3.0 * p->D + 0.5);", T + "test_solute_and_heat_modes_decay_at_the_diffusivity"),
    ("heat rate with 2 alpha", "double s1t = 1.0 / (3.0 * p->alpha / heat_sub(p) + 0.5);",
     "double s1t = 1.0 / (6.0 * p->alpha / heat_sub(p) + 0.5);", T + "test_solute_and_heat_modes_decay_at_the_diffusivity"),
    ("flow second moments relaxed at 1", "double s[9] = {1.0, 1.0, 1.0, s2, s2, s2, 1.0, 1.0, 1.0};",
     "double s[9] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0};", T + "test_taylor_green_decay_with_two_time_scaling"),
    ("coupling source with 1 - phi^2 once", "double Q = ph * om - p->lambda * (theta + p->Mcinf * U) * om * om;",
     "double Q = ph * om - p->lambda * (theta + p->Mcinf * U) * om;", T + "test_undercooled_planar_front_speed"),
    ("heat advection with theta instead of H", "double Hux = H * ux, Huy = H * uy;",
     "double Hux = theta * ux, Huy = theta * uy;", TT + "test_cde_equilibrium_moment_conditions"),
    ("heat advection without 1/cs^2", "out[i] = W5[i] * theta + W5[i] * (3.0 * cu);",
     "out[i] = W5[i] * theta + W5[i] * cu;", T + "test_advected_mode_keeps_the_diffusivity"),
    ("solute rest population with w0", "out[0] = C + (W5[0] - 1.0) * qU;", "out[0] = C + W5[0] * qU;",
     TC + "test_solute_free_melt_stays_free_under_a_moving_front"),
    ("seed width without sqrt 2", "double ph = tanh((p->seed_R - d) / (sqrt(2.0) * p->W0));",
     "double ph = tanh((p->seed_R - d) / p->W0);", T + "test_seed_profile_is_the_stationary_interface"),
    ("force fraction of the liquid", "double qt = 0.5 * (1.0 - phi);", "double qt = 0.5 * (1.0 + phi);",
     T + "test_diffuse_solid_brakes_the_flow"),
    ("forcing without (1 - S/2)", "acc += ((i == j ? 1.0 : 0.0) - 0.5 * L9[i * 9 + j]) * F[j];",
     "acc += (i == j ? 1.0 : 0.0) * F[j];", T + "test_diffuse_solid_brakes_the_flow"),
    ("pressure with the rest population", "if (i) rest += h[i];", "rest += h[i];",
     T + "test_uniform_channel_flow_is_steady"),
    ("corner walls from the x neighbour only", "int yf = y < 1 ? 1 : (y > s->ny - 2 ? s->ny - 2 : y);",
     "int yf = y;", T + "test_channel_conserves_mass_past_an_off_centre_solid"),
    ("free slip keeps the transverse velocity", "                ub[0] = uf[0];\n                ub[1] = 0.0;",
     "                ub[0] = uf[0];\n                ub[1] = uf[1];",
     T + "test_channel_conserves_mass_past_an_off_centre_solid"),
    ("outflow pressure from the neighbour", "ub[1] = (y == 0 || y == s->ny - 1) ? 0.0 : uf[1];\n                pb = 0.0;",
     "ub[1] = (y == 0 || y == s->ny - 1) ? 0.0 : uf[1];\n                pb = pf;",
     T + "test_channel_conserves_mass_past_an_off_centre_solid"),
    ("inflow velocity in main-step units", "ub[0] = s->p.u_in_x / s->p.n_sub;", "ub[0] = s->p.u_in_x;",
     T + "test_uniform_channel_flow_is_steady"),
    ("solid weight (1 - phi)/2 in the reductions", "double w = 0.5 * (1.0 + s->phi[x]);",
     "double w = 0.5 * (1.0 - s->phi[x]);", TC + "test_force_and_torque_balance_the_fluid_momentum"),
    ("viscosity not rescaled by N", "double nu_sub = p->nu / (double)p->n_sub;",
     "double nu_sub = p->nu;", T + "test_taylor_green_decay_with_two_time_scaling"),
    ("h(phi)/2 dropped from g_0^eq", "out[0] = W5[0] * theta - 0.5 * hp;",
     "out[0] = W5[0] * theta;", TT + "test_cde_equilibrium_moment_conditions"),
    ("sign of Mc_inf U", "p->lambda * (theta + p->Mcinf * U)", "p->lambda * (theta - p->Mcinf * U)",
     T + "test_undercooled_planar_front_speed"),
    ("U without 1/(1-k)", "s->U[x] = (2.0 * C / (1.0 + p->k - (1.0 - p->k) * ph) - 1.0) / (1.0 - p->k);",
     "s->U[x] = (2.0 * C / (1.0 + p->k - (1.0 - p->k) * ph) - 1.0);",
     T + "test_solute_and_heat_modes_decay_at_the_diffusivity"),
    ("anisotropy strength", "4.0 * eps / (1.0 - 3.0 * eps) * sum_n4", "3.0 * eps / (1.0 - 3.0 * eps) * sum_n4",
     TT + "test_anisotropy_matches_angle_form"),
    ("sign of N in the local gradient", "double nx = -3.0 * s1 * (m1x + W2t * Nx);",
     "double nx = -3.0 * s1 * (m1x - W2t * Nx);",
     TT + "test_local_gradient_inverts_its_defining_relation"),
    ("pressure coefficient", "(u[0] * u[0] + u[1] * u[1]) / (2.0 * cs2)", "(u[0] * u[0] + u[1] * u[1]) / cs2",
     T + "test_uniform_channel_flow_is_steady"),
    ("velocity term of n^eq", "out[i] = W5[i] * qU + W5[i] * (3.0 * cu);", "out[i] = W5[i] * qU + W5[i] * cu;",
     TT + "test_cde_equilibrium_moment_conditions"),
    ("tip interpolation index", "best = (j - 1) + prev / (prev - v);", "best = j + prev / (prev - v);",
     T + "test_tip_of_a_parabolic_finger"),
    ("transposed D2Q5 Lambda", "acc += Minv[i * n + k] * s[k] * M[k * n + j];",
     "acc += Minv[j * n + k] * s[k] * M[k * n + i];", TT + "test_d2q5_lambda_equals_printed_matrix"),
    ("restart drops the first-moment remainder",
     "3.0 * W5[i] * (C5X[i] * (V[0] - Vo[0]) + C5Y[i] * (V[1] - Vo[1]))",
     "3.0 * W5[i] * (C5X[i] * V[0] + C5Y[i] * V[1])",
     TR + "test_restart_at_own_fields_with_both_flags_changes_nothing"),
    ("restart drops the rates", "s->Q_prev[id] = Q - (Qo - s->Q_prev[id]);", "s->Q_prev[id] = Q;",
     TR + "test_restart_at_own_fields_with_both_flags_changes_nothing"),
    ("anti-trapping current dropped", JAT, "double c = 0.0;", TC + "test_planar_alloy_front_does_not_trap_solute[2]"),
    ("anti-trapping without 1/(2 sqrt 2)", JAT, JAT.replace("-1.0 / (2.0 * sqrt(2.0))", "-1.0"),
     TC + "test_planar_alloy_front_does_not_trap_solute[2]"),
    ("sign of the anti-trapping current", JAT, JAT.replace("-1.0 / (2.0", "1.0 / (2.0"),
     TC + "test_planar_alloy_front_does_not_trap_solute[2]"),
    ("anti-trapping with W0^2", JAT, JAT.replace("p->W0 *", "p->W0 * p->W0 *"),
     TC + "test_planar_alloy_front_does_not_trap_solute[2]"),
    ("anti-trapping without its 1 + (1-k)U factor", JAT, JAT.replace("(1.0 + (1.0 - p->k) * U) * ", ""),
     TC + "test_solute_free_melt_stays_free_under_a_moving_front[2]"),
    ("anti-trapping factor 1 + U", JAT, JAT.replace("(1.0 + (1.0 - p->k) * U)", "(1.0 + U)"),
     TC + "test_solute_free_melt_stays_free_under_a_moving_front[2]"),
    ("sign of the torque", "T -= rx * Fb[1] - ry * Fb[0];", "T += rx * Fb[1] - ry * Fb[0];",
     TC + "test_force_and_torque_balance_the_fluid_momentum"),
    ("torque about the origin", "double rx = (x % s->nx) - cx, ry = (x / s->nx) - cy;",
     "double rx = (x % s->nx), ry = (x / s->nx);", TC + "test_force_and_torque_balance_the_fluid_momentum"),
    ("torque with transposed cross product", "T -= rx * Fb[1] - ry * Fb[0];", "T -= rx * Fb[0] - ry * Fb[1];",
     TC + "test_force_and_torque_balance_the_fluid_momentum"),
]


SRC3 = os.path.join(ROOT, "oracle", "dlb3_oracle.c")
T3 = "tests/test_oracle_3d.py::"
JAT3 = "double c = -1.0 / (2.0 * sqrt(2.0)) * p->W0 * (1.0 + (1.0 - p->k) * U) * dphi / gn;"
# mistakes planted in the 3-D oracle (dlb3_oracle.c)
MUTATIONS_3D = [
    ("3-D: lattice sound speed 1/3 in s1", "return 1.0 / (as * as * p->W0 * p->W0 / (p->tau0 * CS2) + 0.5);",
     "return 1.0 / (3.0 * as * as * p->W0 * p->W0 / p->tau0 + 0.5);",
     T3 + "test_phase_field_mode_decay_with_fixed_anisotropy"),
    ("3-D: heat rate without 1/cs^2", "static double s1_heat(const o3_params* p) { return 1.0 / (p->alpha / CS2 + 0.5); }",
     "static double s1_heat(const o3_params* p) { return 1.0 / (3.0 * p->alpha + 0.5); }",
     T3 + "test_diffusion_mode_decays_at_the_diffusivity"),
    ("3-D: plain streaming for phi", "(s->pf[o + src] - s->f[o + d]) / s->a2[src];", "(s->pf[o + src] - s->f[o + d]);",
     T3 + "test_phase_field_mode_decay_with_fixed_anisotropy"),
    ("3-D flow: second moments relaxed at 1", "for (int q = 0; q < 19; ++q) second[q] = (q >= 4 && q <= 9);",
     "for (int q = 0; q < 19; ++q) second[q] = 0;", T3 + "test_shear_wave_decays_at_nu"),
    ("3-D: heat equilibrium with cs^2 = 1/3", "(CX[i] * H * u[0] + CY[i] * H * u[1] + CZ[i] * H * u[2]) / CS2;",
     "(CX[i] * H * u[0] + CY[i] * H * u[1] + CZ[i] * H * u[2]) * 3.0;", T3 + "test_advected_heat_mode_keeps_alpha_and_u"),
    ("3-D: anisotropy strength", "out[1 + a] = g2 * as * (4.0 * eps * dsum);", "out[1 + a] = g2 * as * (3.0 * eps * dsum);",
     T3 + "test_torque_vector_is_the_gradient_of_a_s"),
    ("3-D: seed width without sqrt 2", "tanh((p->seed_R - d) / (sqrt(2.0) * p->W0));",
     "tanh((p->seed_R - d) / p->W0);", T3 + "test_seed_profile_is_the_stationary_interface"),
    ("3-D: free slip keeps the transverse velocity",
     "                } else {\n                    ub[0] = uf[0];\n                    ub[1] = ywall ? 0.0 : uf[1];",
     "                } else {\n                    ub[0] = uf[0];\n                    ub[1] = uf[1];",
     T3 + "test_channel_conserves_mass_past_an_off_centre_solid"),
    ("3-D: outflow pressure from the neighbour", "                    pb = 0.0;", "                    pb = pf;",
     T3 + "test_channel_conserves_mass_past_an_off_centre_solid"),
    ("3-D: sign of G^phi", "G[i] = -W7[i] * (CX[i] * lg[4] + CY[i] * lg[5] + CZ[i] * lg[6]) / a2;",
     "G[i] = W7[i] * (CX[i] * lg[4] + CY[i] * lg[5] + CZ[i] * lg[6]) / a2;",
     T3 + "test_front_undulation_relaxes_with_anisotropic_stiffness"),
    ("3-D: sign of U grad q", "U * (-0.5 * gx)", "U * (0.5 * gx)",
     T3 + "test_uniform_U_and_theta_are_steady_across_a_still_front"),
    ("3-D: solute rate without 1 - k",
     "static double s1_solute(const o3_params* p) { return 1.0 / (p->D * (1.0 - p->k) / CS2 + 0.5); }",
     "static double s1_solute(const o3_params* p) { return 1.0 / (p->D / CS2 + 0.5); }",
     T3 + "test_diffusion_mode_decays_at_the_diffusivity"),
    ("3-D: h(phi)/2 dropped from g_0^eq", "o[0] = W7[0] * theta - 0.5 * h_of(phi, quintic);",
     "o[0] = W7[0] * theta;", T3 + "test_uniform_U_and_theta_are_steady_across_a_still_front"),
    ("3-D: coupling source with 1 - phi^2 once", "double Q = ph * om - p->lambda * (th + p->Mcinf * U) * om * om;",
     "double Q = ph * om - p->lambda * (th + p->Mcinf * U) * om;", T3 + "test_undercooled_planar_front_speed"),
    ("3-D: anti-trapping current dropped", JAT3, "double c = 0.0;",
     TC + "test_planar_alloy_front_does_not_trap_solute[3]"),
    ("3-D: anti-trapping without 1/(2 sqrt 2)", JAT3, JAT3.replace("-1.0 / (2.0 * sqrt(2.0))", "-1.0"),
     TC + "test_planar_alloy_front_does_not_trap_solute[3]"),
    ("3-D: sign of the anti-trapping current", JAT3, JAT3.replace("-1.0 / (2.0", "1.0 / (2.0"),
     TC + "test_planar_alloy_front_does_not_trap_solute[3]"),
    ("3-D: anti-trapping with W0^2", JAT3, JAT3.replace("p->W0 *", "p->W0 * p->W0 *"),
     TC + "test_planar_alloy_front_does_not_trap_solute[3]"),
    ("3-D: anti-trapping without its 1 + (1-k)U factor", JAT3, JAT3.replace("(1.0 + (1.0 - p->k) * U) * ", ""),
     TC + "test_solute_free_melt_stays_free_under_a_moving_front[3]"),
    ("3-D: anti-trapping factor 1 + U", JAT3, JAT3.replace("(1.0 + (1.0 - p->k) * U)", "(1.0 + U)"),
     TC + "test_solute_free_melt_stays_free_under_a_moving_front[3]"),
]


def _run_mutant(workdir, dim, label, old, new, pin):
    """Build the oracle with one planted mistake and run its pin against it in
    a child pytest; returns (child's return code, the tail of its output)."""
    src_path, env_var = (SRC, "DLB_ORACLE_LIB") if dim == 2 else (SRC3, "DLB3_ORACLE_LIB")
    src = open(src_path).read()
    if src.count(old) != 1:
        return None, f"mutation anchor not unique/found: {old!r}"
    os.makedirs(workdir, exist_ok=True)
    mut_c = os.path.join(workdir, "mutant.c")
    lib = os.path.join(workdir, "libmutant.so")
    with open(mut_c, "w") as fh:
        fh.write(src.replace(old, new))
    inc = ["-I", os.path.dirname(SRC)] if dim == 2 else []
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", *inc,
                    "-o", lib, mut_c, "-lm"], check=True)
    # the children run side by side, one OpenMP thread each
    env = dict(os.environ, **{env_var: lib, "OMP_NUM_THREADS": "1"})
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", pin],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return r.returncode, r.stdout[-2000:]


@pytest.fixture(scope="module")
def mutant_runs(tmp_path_factory):
    """Every planted mistake, built and run against its pin in parallel child
    processes; keyed by (dimension, label)."""
    cases = [(2, *m) for m in MUTATIONS] + [(3, *m) for m in MUTATIONS_3D]
    base = tmp_path_factory.mktemp("mutants")
    workers = max(1, min(8, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        futs = {(dim, label): ex.submit(_run_mutant, os.path.join(base, f"m{i:03d}"), dim, label, old, new, pin)
                for i, (dim, label, old, new, pin) in enumerate(cases)}
        return {key: fut.result() for key, fut in futs.items()}


@pytest.mark.parametrize("label,old,new,pin", MUTATIONS_3D, ids=[m[0] for m in MUTATIONS_3D])
def test_pin_catches_planted_mistake_3d(mutant_runs, label, old, new, pin):
    rc, out = mutant_runs[(3, label)]
    assert rc is not None, out
    assert rc != 0, f"pin {pin} did not catch: {label}\n{out}"


@pytest.mark.parametrize("label,old,new,pin", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_planted_mistake(mutant_runs, label, old, new, pin):
    rc, out = mutant_runs[(2, label)]
    assert rc is not None, out
    assert rc != 0, f"pin {pin} did not catch: {label}\n{out}"
