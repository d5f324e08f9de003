"""The oracle's pins catch the mistakes they are written against.

Each case plants one plausible mistake in a copy of the oracle's source,
builds it on the CPU, and runs the pins named for it against that build in a
fresh process (the oracle wrapper loads the build that JZO_LIB names).  The
named pins must fail; the unpatched source built the same way must pass them
all.  The mistakes, by part of Sec. 3:
  * closure: Cv for Cp or Pr_t for Pr in the heat conduction of Eq. (q_mod),
    the sign of q, the -2/3 div u part of Eq. (tau_mod), the viscous work of
    Eq. (vec-les), the Sutherland exponent, Cs once instead of squared, the
    Jacobian dropped from the chain-rule gradients;
  * inviscid part: the kinetic energy in the equation of state, the metric
    index of the contravariant flux;
  * dissipation (closing paragraph): the second-difference branch, its
    clamp, a fixed fourth-difference coefficient, a one-sided sensor or a
    wrong sensor denominator, the third-difference coefficient, the sound
    speed dropped from the spectral radius, the anisotropy exponent;
  * time integration: a stage coefficient, the sound speed dropped from the
    CFL radius;
  * boundaries: the sign of the incoming Riemann invariant, the side that
    supplies entropy, the divisor of the centreline average.
These pins compare with closed forms, exact solutions and invariants, never
with the second NumPy coding of the oracle.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "jetles_oracle.cpp")
PIN_FILES = [os.path.join(ROOT, "tests", f) for f in
             ("test_oracle_closure_pins.py", "test_oracle_pins.py", "test_oracle_bc_pins.py")]

KAPPA = "const double kap = cp * mu / P.prandtl + cp * mut / P.prandtl_t;"
WORK = ("EV[c][4] = (e + p) * uu[c] - (uu[0] * tau[0][c] + uu[1] * tau[1][c] + uu[2] * tau[2][c]"
        " - qh[c]);")
EPS4 = "const double eps4 = std::max(0.0, P.k4 - eps2);"
HEAT = "test_heat_conduction_rate_of_a_temperature_wave"
LONG = "test_longitudinal_wave_has_four_thirds_viscosity"
SHEAR = "test_viscous_work_of_a_shear_wave_on_a_uniform_stream"
SOD = "test_sod_shock_tubes_converge_to_the_exact_solution"
SPIKE = "test_dissipation_face_flux_of_a_pressure_spike"
SHEAR_RK = "test_shear_wave_decay_factor_wide_viscous_stencil_and_rk_polynomial"
ENTROPY = "test_entropy_wave_convection_and_fourth_difference_dissipation"
SUTHERLAND = "test_sutherland_reference_and_textbook_ratio"
SMAGORINSKY = "test_smagorinsky_closed_form_on_sine_shear"
VORTEX = "test_isentropic_vortex_short_time_and_second_order"
FREESTREAM = "test_freestream_roundoff_on_wavy_grid_with_tl_metrics"
CFL = "test_cfl_dt_special_case_and_viscous_limit_on_jet_box"
INVARIANTS = "test_subsonic_far_field_carries_the_riemann_invariants"
FIXED_POINT = "test_free_stream_is_a_fixed_point_of_the_far_field"
AXIS = "test_centreline_takes_the_ordered_azimuthal_mean_of_the_adjacent_ring"

# name: (source fragment, its mistaken version, pins that must fail)
MUTANTS = {
    "cv_for_cp": (KAPPA, "const double kap = (cp / gam) * mu / P.prandtl + (cp / gam) * mut / P.prandtl_t;",
                  [HEAT]),
    "prandtl_swapped": (KAPPA, "const double kap = cp * mu / P.prandtl_t + cp * mut / P.prandtl;",
                        [HEAT, "test_heat_conduction_subgrid_uses_turbulent_prandtl_number"]),
    "heat_flux_sign": ("qh[c] = -kap * f.g[(9 + c) * N + n];", "qh[c] = kap * f.g[(9 + c) * N + n];", [HEAT]),
    "div_u_dropped": ("(a == c ? 2.0 / 3.0 * div : 0.0)", "(a == c ? 0.0 * div : 0.0)", [LONG]),
    "div_u_sign": ("(a == c ? 2.0 / 3.0 * div : 0.0)", "(a == c ? -2.0 / 3.0 * div : 0.0)", [LONG]),
    "work_dropped": (WORK, "EV[c][4] = (e + p) * uu[c] - (- qh[c]);", [SHEAR]),
    "work_sign": (WORK, "EV[c][4] = (e + p) * uu[c] - (-(uu[0] * tau[0][c] + uu[1] * tau[1][c]"
                        " + uu[2] * tau[2][c]) - qh[c]);", [SHEAR]),
    "eps2_dropped": ("const double dface = sg * (eps2 * (Q[nR] - Q[nL]) - eps4 * d3);",
                     "const double dface = sg * (0.0 * (Q[nR] - Q[nL]) - eps4 * d3);", [SOD, SPIKE]),
    "clamp_dropped": (EPS4, "const double eps4 = P.k4 - eps2;", [SPIKE]),
    "eps4_fixed": (EPS4, "const double eps4 = P.k4;", [SPIKE]),
    "sensor_one_sided": ("const double eps2 = P.k2 * std::max(f.nu[d * N + nL], f.nu[d * N + nR]);",
                         "const double eps2 = P.k2 * f.nu[d * N + nL];", [SPIKE]),
    "sensor_denominator": ("/ (pp + 2.0 * f.p[n] + pm);", "/ (pp + f.p[n] + pm);", [SPIKE]),
    "sutherland_exponent": ("mu_inf * std::pow(T, 1.5)", "mu_inf * std::pow(T, 1.0)", [SUTHERLAND]),
    "smagorinsky_cs_once": ("(P.cs * delta) * (P.cs * delta) * smag", "(P.cs * delta) * delta * smag",
                            [SMAGORINSKY]),
    "gradient_without_jacobian": ("f.g[(3 * s + a) * N + n] = J * acc;", "f.g[(3 * s + a) * N + n] = acc;",
                                  [SHEAR_RK]),
    "kinetic_energy_whole": ("const double p = (gam - 1.0) * (q[4 * N + n] - 0.5 * rho * (u * u + v * v + w * w));",
                             "const double p = (gam - 1.0) * (q[4 * N + n] - rho * (u * u + v * v + w * w));",
                             [ENTROPY, VORTEX]),
    "flux_metric_transposed": ("acc += m[(3 * d + c) * N + n] * EV[c][v];",
                               "acc += m[(3 * c + d) * N + n] * EV[c][v];", [FREESTREAM]),
    "lambda_without_sound": ("f.lam[d * N + n] = std::fabs(U) + f.a[n] * std::fabs(J)"
                             " * std::sqrt(sx * sx + sy * sy + sz * sz);",
                             "f.lam[d * N + n] = std::fabs(U);", [ENTROPY]),
    "anisotropy_exponent": ("std::pow(f.lam[e2 * N + n] / ld, P.tv_alpha)", "std::pow(f.lam[e2 * N + n] / ld, 1.0)",
                            [ENTROPY]),
    "third_difference": ("(Q[nRR] - Q[nLL]) - 3.0 * (Q[nR] - Q[nL])", "(Q[nRR] - Q[nLL]) - 2.0 * (Q[nR] - Q[nL])",
                         [ENTROPY]),
    "rk_stage_coefficient": ("p->rk_alpha[1] = 1.0 / 6.0;", "p->rk_alpha[1] = 1.0 / 5.0;", [SHEAR_RK, ENTROPY]),
    "cfl_without_sound": ("sum += std::fabs(J * (sx * u + sy * v + sz * w)) + a * std::fabs(J)"
                          " * std::sqrt(sx * sx + sy * sy + sz * sz);",
                          "sum += std::fabs(J * (sx * u + sy * v + sz * w));", [CFL]),
    "incoming_invariant_sign": ("const double rm = une - 2.0 * ae / (g - 1.0);",
                                "const double rm = une + 2.0 * ae / (g - 1.0);", [INVARIANTS, FIXED_POINT]),
    "entropy_side": ("const bool out = unb > 0.0;", "const bool out = unb < 0.0;", [INVARIANTS]),
    "axis_mean_divisor": ("acc[v] /= (double)b.n[2];", "acc[v] /= (double)(b.n[2] - 1);", [AXIS]),
}


def _build(src_text: str, out: str) -> str:
    cpp = out[:-3] + ".cpp"
    with open(cpp, "w") as f:
        f.write(src_text)
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", cpp, "-o", out])
    return out


def _run_pins(lib: str, names):
    env = dict(os.environ, JZO_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", *PIN_FILES, "-q", "-p", "no:cacheprovider",
                        "-k", " or ".join(names)], cwd=ROOT, env=env, capture_output=True, text=True)
    return r.returncode, r.stdout + r.stderr


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    d = tmp_path_factory.mktemp("oracle_mutants")
    src = open(SRC).read()
    jobs = {"unpatched": src}
    for name, (old, new, _) in MUTANTS.items():
        assert src.count(old) == 1, f"{name}: the fragment to patch is not unique in the oracle source"
        jobs[name] = src.replace(old, new)
    with ThreadPoolExecutor(max_workers=4) as ex:
        futs = {k: ex.submit(_build, v, str(d / f"{k}.so")) for k, v in jobs.items()}
        return {k: f.result() for k, f in futs.items()}


@pytest.fixture(scope="module")
def results(builds):
    """Every build against the pins named for its mistake (the unpatched one
    against all of them), four processes at a time."""
    names = sorted({p for _, _, pins in MUTANTS.values() for p in pins})
    todo = {"unpatched": names}
    todo.update({k: pins for k, (_, _, pins) in MUTANTS.items()})
    with ThreadPoolExecutor(max_workers=4) as ex:
        futs = {k: ex.submit(_run_pins, builds[k], v) for k, v in todo.items()}
        return {k: f.result() for k, f in futs.items()}


def test_unpatched_build_passes_the_pins(results):
    rc, out = results["unpatched"]
    assert rc == 0, out[-3000:]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(results, name):
    rc, out = results[name]
    assert rc == 1, f"{name}: expected failing pins, pytest returned {rc}\n{out[-3000:]}"
    failed = [line for line in out.splitlines() if line.startswith("FAILED ")]
    for pin in MUTANTS[name][2]:
        assert any(f"::{pin}" in line for line in failed), f"{name}: {pin} did not fail\n{out[-3000:]}"
