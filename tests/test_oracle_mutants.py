"""Planted mistakes in the oracle (CPU only). Each mutant is a copy of the
oracle's C source with one plausible error: a sign, a dropped or swapped
term, a wrong weight or step, an off-by-one in the random-number generator
or the swarm update. It is built on its own and the pin tests run against
it in a child process; every mutant must fail at least one pin. This checks
that the pins constrain each part of the oracle, not only its overall
shape. Nothing here touches the GPU library."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# name: (text in the oracle source, replacement); each text occurs once
MUTANTS = {
    # equations of motion (Background, eqs. cr3bp:x-z)
    "coriolis_x_sign": ("fma(2.0, vy, x)));", "fma(-2.0, vy, x)));"),
    "coriolis_y_sign": ("fma(-cs, y, fma(-2.0, vx, y));", "fma(-cs, y, fma(2.0, vx, y));"),
    "second_primary_position": ("const double d2 = x - mu1;", "const double d2 = x - mu;"),
    "first_primary_mass": ("const double c1 = mu1 * (D2 * R);", "const double c1 = mu * (D2 * R);"),
    "z_acceleration_term": ("f[5] = -(cs * z);", "f[5] = -(c1 * z);"),
    # classical RK4
    "rk4_second_stage_weight": ("double a = fma(2.0, k2[d], k1[d]);",
                                "double a = fma(1.0, k2[d], k1[d]);"),
    "rk4_last_stage_step": ("for (d = 0; d < 6; d++) s[d] = fma(h, k3[d], X[d]);",
                            "for (d = 0; d < 6; d++) s[d] = fma(h2, k3[d], X[d]);"),
    # observation schedule and partial steps
    "schedule_truncates": ("nn = (int64_t)floor(q + 0.5);", "nn = (int64_t)floor(q);"),
    "partial_step_moves_the_grid": ("if (T->tau[k] != 0.0) orc_rk4_step(P->mu, T->tau[k], S);",
                                    "if (T->tau[k] != 0.0) orc_rk4_step(P->mu, T->tau[k], X);"),
    # measurement model and cost (eqs. rel:pos, meas:function, b:total, total:cost)
    "azimuth_residual_sign": ("na = fma(sa, rx, -(ca * ry));", "na = fma(sa, rx, (ca * ry));"),
    "elevation_sin_cos_swapped": (
        "*db = atan2(fma(sb, rxy, -(cb * rz)), fma(cb, rxy, sb * rz));",
        "*db = atan2(fma(cb, rxy, -(sb * rz)), fma(sb, rxy, cb * rz));"),
    "weight_is_one_over_sigma": ("T->w = 1.0 / (P->sigma * P->sigma);", "T->w = 1.0 / P->sigma;"),
    "elevation_term_dropped": ("e = T->w * fma(da, da, db * db);", "e = T->w * (da * da);"),
    "paper_cost_not_squared": ("            J = fma(e, e, J);", "            J = J + e;"),
    # Philox4x64-10 and its uniform doubles
    "philox_nine_rounds": ("for (r = 0; r < 10; r++) {", "for (r = 0; r < 9; r++) {"),
    "philox_weyl_constant": ("k1 += 0xBB67AE8584CAA73BULL;", "k1 += 0xBB67AE8584CAA73AULL;"),
    "uniform_drops_a_bit": ("return (double)(w >> 11) * 0x1.0p-53;",
                            "return (double)(w >> 12) * 0x1.0p-53;"),
    # Algorithm 1
    "init_box_width": ("x[6 * i + d] = S->lo[d] + (S->hi[d] - S->lo[d]) * u[d];",
                       "x[6 * i + d] = S->lo[d] + (S->hi[d] + S->lo[d]) * u[d];"),
    "social_term_uses_pbest": ("a2[d] * (g[d] - xi);", "a2[d] * (g[d] - p[6 * i + d]);"),
    "inertia_on_position": ("S->omega * v[6 * i + d]", "S->omega * x[6 * i + d]"),
    "one_coefficient_for_both_terms": ("a2[d] = S->eta2 * u01(u[1]);",
                                       "a2[d] = S->eta2 * u01(u[0]);"),
    "counter_words_swapped": ("c[0] = (uint64_t)n; c[1] = (uint64_t)i;",
                              "c[0] = (uint64_t)i; c[1] = (uint64_t)n;"),
}

# mutants of the sensitivity and variant code, run against those pins
MUTANTS_SENS_VARIANTS = {
    # tangent of the RK4 map and residual Jacobians
    "jacobian_coriolis_sign": ("A[6 * 3 + 4] = 2.0;", "A[6 * 3 + 4] = -2.0;"),
    "jacobian_power": ("e2 = 3.0 * mu / pow(r2, 5);", "e2 = 3.0 * mu / pow(r2, 3);"),
    "tangent_stage_weight": ("const double wt[4] = {1.0, 2.0, 2.0, 1.0};",
                             "const double wt[4] = {1.0, 2.0, 1.0, 1.0};"),
    "azimuth_gradient_sign": ("ga[0] = rho[1] / rxy2;", "ga[0] = -rho[1] / rxy2;"),
    "elevation_gradient_sign": ("gb[2] = -rxy / r2;", "gb[2] = rxy / r2;"),
    # range measurement
    "range_weight_is_one_over_sigma": (
        "T->wr = P->ranges ? 1.0 / (P->sigma_range * P->sigma_range) : 0.0;",
        "T->wr = P->ranges ? 1.0 / P->sigma_range : 0.0;"),
    "range_residual_sign": ("const double dr = T->ranges[k] - range_of(rho);",
                            "const double dr = T->ranges[k] + range_of(rho);"),
    # extended-precision residuals (the refinement's accuracy reference)
    "ld_elevation_residual_sign": ("db = (ld)P->angles[2 * k + 1] - asinl(rz / rn);",
                                   "db = (ld)P->angles[2 * k + 1] + asinl(rz / rn);"),
    "ld_residual_weight": ("r[R * k] = (double)(da * is);", "r[R * k] = (double)(da / is);"),
    "ld_range_residual_sign": ("if (P->ranges) dr = (ld)P->ranges[k] - rn;",
                               "if (P->ranges) dr = rn - (ld)P->ranges[k];"),
    # constriction, grid initialisation, per-dimension coefficients, Algorithm 2
    "constriction_formula": ("return 2.0 / fabs(2.0 - phi - sqrt(phi * phi - 4.0 * phi));",
                             "return 2.0 / fabs(2.0 - phi - sqrt(phi * phi - 2.0 * phi));"),
    "grid_levels_off_by_one": ("if (G / b * (b + 1) > m) break;",
                               "if (G / b * (b + 1) >= m) break;"),
    "per_dimension_word": ("a1[d] = S->eta1 * u01(u[2 * d]);", "a1[d] = S->eta1 * u01(u[d]);"),
    "algorithm2_lag": ("orc_tolerance_met(hist[n], hist[n - S->tol_lag], S->tol))",
                       "orc_tolerance_met(hist[n], hist[n - S->tol_lag + 1], S->tol))"),
}

CHILD = """
import sys
sys.path.insert(0, {root!r})
import oracle
oracle._LIB = {lib!r}
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", *{tests!r}]))
"""


def run_mutant(tmp_path, name, old, new, test_files):
    import oracle
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, f"{name}: the text to mutate must occur exactly once"
    mutant = tmp_path / "orc_mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = str(tmp_path / "liborc_mutant.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", lib, str(mutant), "-lm"], check=True, capture_output=True)
    env = dict(os.environ, OMP_NUM_THREADS="4")
    code = CHILD.format(root=ROOT, lib=lib,
                        tests=[os.path.join(ROOT, "tests", t) for t in test_files])
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=600)
    # 1: a pin failed; a negative code: the mutant crashed the run. 0 would
    # mean every pin passed with the mistake in place.
    assert r.returncode == 1 or r.returncode < 0, (name, r.returncode, r.stdout[-2000:])
    failed = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    print(name, "->", failed[:1])


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, name):
    run_mutant(tmp_path, name, *MUTANTS[name], ["test_oracle_pins.py"])


@pytest.mark.parametrize("name", sorted(MUTANTS_SENS_VARIANTS))
def test_sensitivity_and_variant_pins_catch_planted_mistake(tmp_path, name):
    run_mutant(tmp_path, name, *MUTANTS_SENS_VARIANTS[name],
               ["test_oracle_sensitivity.py", "test_oracle_variants.py"])
