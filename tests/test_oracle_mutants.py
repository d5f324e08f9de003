"""The closure and shock pins catch the mistakes they are written against.

Each case plants one plausible mistake in a copy of the oracle's source
(Sec. 3: Cv for Cp or Pr_t for Pr in the heat conduction of Eq. (q_mod), the
sign of q, the -2/3 div u part of Eq. (tau_mod), the viscous work of
Eq. (vec-les); the second-difference branch of the dissipation and its
clamp, closing paragraph), builds it on the CPU, and runs the pins of
tests/test_oracle_closure_pins.py against it in a fresh process (the oracle
wrapper loads the build that JZO_LIB names).  The pins named for the mistake
must fail; the unpatched source built the same way must pass them all.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "jetles_oracle.cpp")
PINS = os.path.join(ROOT, "tests", "test_oracle_closure_pins.py")

KAPPA = "const double kap = cp * mu / P.prandtl + cp * mut / P.prandtl_t;"
WORK = ("EV[c][4] = (e + p) * uu[c] - (uu[0] * tau[0][c] + uu[1] * tau[1][c] + uu[2] * tau[2][c]"
        " - qh[c]);")
EPS4 = "const double eps4 = std::max(0.0, P.k4 - eps2);"
HEAT = "test_heat_conduction_rate_of_a_temperature_wave"
LONG = "test_longitudinal_wave_has_four_thirds_viscosity"
SHEAR = "test_viscous_work_of_a_shear_wave_on_a_uniform_stream"
SOD = "test_sod_shock_tubes_converge_to_the_exact_solution"
SPIKE = "test_dissipation_face_flux_of_a_pressure_spike"

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
}


def _build(src_text: str, out: str) -> str:
    cpp = out[:-3] + ".cpp"
    with open(cpp, "w") as f:
        f.write(src_text)
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", cpp, "-o", out])
    return out


def _run_pins(lib: str, names):
    env = dict(os.environ, JZO_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", PINS, "-q", "-p", "no:cacheprovider",
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
