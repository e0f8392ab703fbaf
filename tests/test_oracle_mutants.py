"""The oracle pins must reject plausible mistakes.

Each case plants one mistake in a private copy of the C oracle (a dropped
term, a flipped sign, a transposed operand, a wrong factor), builds it, and
runs the pin suite against it in a subprocess; the suite has to fail.  The
mistakes in the relaxation alternatives (or_solve_variant) and in the
stagnation stop are checked against their own pins
(tests/test_oracle_variants.py, tests/test_oracle_floor.py).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dr_oracle.c")

MUTANTS = {
    "force_sign": ("f[3 * j + c] += fc;", "f[3 * j + c] -= fc;"),
    "strain_dropped_one": ("double eps = l / L0[k] - 1.0;", "double eps = l / L0[k];"),
    "exp_law_dropped_term": ("*T = o->EA * (e - 1.0) / o->B;", "*T = o->EA * e / o->B;"),
    "exp_branch_threshold": ("if (o->law == OR_EXP && eps >= 0.0) {\n        double e", "if (o->law == OR_EXP && eps >= 0.05) {\n        double e"),
    "stress_no_jacobian": ("sigma[k] = tau[k] / (J * V0);", "sigma[k] = tau[k] / V0;"),
    "affine_map_transposed": ("y[i] = F[3 * i + 0] * X[0] + F[3 * i + 1] * X[1] + F[3 * i + 2] * X[2];",
                              "y[i] = F[i] * X[0] + F[3 + i] * X[1] + F[6 + i] * X[2];"),
    "damping_sign": ("a[3 * p + k] = -(f[3 * p + k] + c * M[p] * v[3 * p + k]) / M[p];",
                     "a[3 * p + k] = -(f[3 * p + k] - c * M[p] * v[3 * p + k]) / M[p];"),
    "timestep_factor": ("double dt = o->alpha * 2.0 / sqrt(gmax);", "double dt = o->alpha * 4.0 / sqrt(gmax);"),
    "gershgorin_factor": ("G[i] += 2.0 * b;", "G[i] += 0.5 * b;"),
    "geometric_stiffness_sign": ("g * ((r == c ? 1.0 : 0.0) - n[r] * n[c])", "g * ((r == c ? 1.0 : 0.0) + n[r] * n[c])"),
    "exp_tangent_factor": ("*kt = o->EA * e;", "*kt = o->EA * e / o->B;"),
    "energy_dropped_term": ("return L0 * o->EA * ((exp(Bb * eps) - 1.0) / Bb - eps) / Bb;",
                            "return L0 * o->EA * ((exp(Bb * eps) - 1.0) / Bb) / Bb;"),
    "residual_includes_boundary": ("if (is_bnd[p]) { B2 += s; continue; }\n        R2 += s;\n        for (int k = 0; k < 3; ++k) a[3 * p + k]",
                                   "R2 += s; if (is_bnd[p]) { B2 += s; continue; }\n        for (int k = 0; k < 3; ++k) a[3 * p + k]"),
    "mass_missing_half_step": ("v[3 * p + k] += 0.5 * dt * a[3 * p + k];\n                x[3 * p + k]",
                               "v[3 * p + k] += dt * a[3 * p + k];\n                x[3 * p + k]"),
}


# mistakes in the relaxation alternatives (or_solve_variant)
VARIANT_MUTANTS = {
    "kinetic_reset_inverted": ("if (KE < KE_prev) {", "if (KE > KE_prev) {"),
    "adaptive_geometric_sign": ("num += kt / L0[k] * nd * nd + T / l * (du2 - nd * nd);",
                                "num += kt / L0[k] * nd * nd - T / l * (du2 - nd * nd);"),
    "adaptive_without_mass": ("den += M[p] * u * u;", "den += u * u;"),
    "damping_work_dropped": ("Wd += cc * M[p] * v[3 * p + k] * v[3 * p + k] * dt;", "Wd += 0.0;"),
}


def _run_mutant(old, new, pins, tmp_path):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old}"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new, 1))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(lib), str(mut), "-lm", "-lpthread"])
    env = dict(os.environ, RVE_ORACLE_LIB=str(lib))
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           os.path.join(ROOT, "tests", pins)], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=600)


# mistakes in the stagnation stop of or_solve
FLOOR_MUTANTS = {
    "stall_never_reset": ("                stall = 0;\n", "\n"),
    "window_off_by_one": ("++stall >= o->stall_checks", "++stall > o->stall_checks"),
    "floor_not_tested": ("R <= ftol && D <= ftol", "D <= ftol"),
    "halving_against_start": ("if (R < 0.5 * Rref) {", "if (R < 0.5 * Rref && n < 0) {"),
}


@pytest.mark.parametrize("name", sorted(FLOOR_MUTANTS))
def test_floor_pins_reject_mutant(name, tmp_path):
    old, new = FLOOR_MUTANTS[name]
    r = _run_mutant(old, new, "test_oracle_floor.py", tmp_path)
    assert r.returncode != 0, f"floor pins accepted mutant {name}:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name", sorted(VARIANT_MUTANTS))
def test_variant_pins_reject_mutant(name, tmp_path):
    old, new = VARIANT_MUTANTS[name]
    r = _run_mutant(old, new, "test_oracle_variants.py", tmp_path)
    assert r.returncode != 0, f"variant pins accepted mutant {name}:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {name}"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new, 1))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(lib), str(mut), "-lm", "-lpthread"])
    env = dict(os.environ, RVE_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"pins accepted mutant {name}:\n{r.stdout[-2000:]}"
