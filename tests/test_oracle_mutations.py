"""The oracle's pins are sensitive: plausible mistakes planted in a copy of
the oracle (a dropped term, a wrong sign, a wrong index, a swapped rule)
make the pin tests fail.  Each mutant is compiled into a temporary
directory and the pins that should catch it are run against it."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "fsl_oracle.c")

MUTANTS = {
    "sixth_order_term": ("+ 4.0 * k_(1, 1, 1) * k_(1, 1, 1);\n    double s222",
                         "+ 2.0 * k_(1, 1, 1) * k_(1, 1, 1);\n    double s222",
                         "test_oracle_collision.py", "brute_force"),
    "inverse_chimera": ("double f0 = k0 * (1.0 - u * u) - 2.0 * u * k1 - k2;",
                        "double f0 = k0 * (1.0 - u * u) - 1.0 * u * k1 - k2;",
                        "test_oracle_collision.py", "identity"),
    "force_shift": ("(j[d] + 0.5 * r * g[d]) / r", "(j[d] + 1.0 * r * g[d]) / r",
                    "test_oracle_collision.py", "momentum"),
    "shear_rate": ("Cs[K(1, 0, 1)] = (1.0 - omega) * C_(1, 0, 1);",
                   "Cs[K(1, 0, 1)] = (1.0 - omega_bulk) * C_(1, 0, 1);",
                   "test_oracle_collision.py", "brute_force or cube"),
    "moving_wall_sign": ("fin[j] = fo[opp(j)] + 6.0 * WT[j]", "fin[j] = fo[opp(j)] - 6.0 * WT[j]",
                         "test_oracle_flow.py", "couette"),
    "laplace_factor": ("p->rho_gas + 6.0 * p->sigma", "p->rho_gas + 3.0 * p->sigma",
                       "test_oracle_flow.py", "cylinder"),
    "flux_weight": ("? 0.5 * (clamp01(L->phi[c]) + clamp01(L->phi[y]))", "? clamp01(L->phi[c])",
                    "test_oracle_flow.py", "channel_film_mass"),
    "flux_index": ("double in = L->f[y * Q + opp(i)], out = fo[i];", "double in = L->f[y * Q + i], out = fo[i];",
                   "test_oracle_flow.py", "tracks_density"),
    "reconstruction": ("fin[j] = feqG[j] + feqG[opp(j)] - fo[opp(j)];",
                       "fin[j] = 2.0 * feqG[j] - fo[opp(j)];",
                       "test_oracle_flow.py", "film or hydrostatic"),
    "normal_side": ("if (nc < -p->normal_tie) recon = 1;", "if (nc > p->normal_tie) recon = 1;",
                    "test_oracle_flow.py", "gravity_driven_film"),
    "no_cancel": ("if (near_fill) {\n            L->cnt[4]++;", "if (0) {\n            L->cnt[4]++;",
                  "test_oracle_conversion.py", "rule_text"),
    "excess_to_liquid": ("if (y >= 0 && L->type[y] == OL_INTERFACE) {\n                recv++;",
                         "if (y >= 0 && L->type[y] != OL_GAS && L->type[y] != OL_SOLID) {\n                recv++;",
                         "test_oracle_conversion.py", "rule_text"),
    "mean_includes_emptying": ("if (mk[y] & MK_TO_GAS) continue;", "if (0) continue;",
                               "test_oracle_conversion.py", "rule_text"),
    "parker_youngs_weight": ("static const double Wpy[3] = {1.0, 2.0, 1.0};",
                             "static const double Wpy[3] = {1.0, 1.0, 1.0};",
                             "test_oracle_geometry.py", "quadratic"),
    "flux_modifier_direction": ("if (cls[c] < cls[y]) in = 0.0;", "if (cls[c] > cls[y]) in = 0.0;",
                                "test_oracle_variants.py", "flux_modifiers_direct"),
    "flux_modifier_class": ("if (has_gas && !has_liq) cls[c] = 0;", "if (has_liq && !has_gas) cls[c] = 0;",
                            "test_oracle_variants.py", "flux_modifiers_direct"),
    "excess_weight_side": ("if (!filled) nc = -nc;", "if (filled) nc = -nc;",
                           "test_oracle_variants.py", "diagonal"),
    "excess_receiver_link": ("excess_weight(L, &L->n[3 * y], opp(i),", "excess_weight(L, &L->n[3 * y], i,",
                             "test_oracle_variants.py", "diagonal"),
    "excess_no_fallback": ("} else if (recv > 0) {\n            L->share[c] = e / recv;",
                           "} else if (0) {\n            L->share[c] = e / recv;",
                           "test_oracle_variants.py", "falls_back"),
    "dem_damping_sign": ("const double gn = -2.0 * meff * lne / p->collision_time;",
                         "const double gn = 2.0 * meff * lne / p->collision_time;",
                         "test_oracle_dem.py", "head_on", "dem_oracle.c"),
    "dem_effective_mass": ("else meff = D->m[a] * D->m[b] / (D->m[a] + D->m[b]);", "else meff = D->m[a];",
                           "test_oracle_dem.py", "head_on", "dem_oracle.c"),
    "dem_contact_point": ("const double la = ra - 0.5 * delta, lb = rb - 0.5 * delta;",
                          "const double la = ra, lb = rb;", "test_oracle_dem.py", "oblique", "dem_oracle.c"),
    "dem_friction_cap": ("lim = p->friction * fabs(fn);", "lim = 2.0 * p->friction * fabs(fn);",
                         "test_oracle_dem.py", "sliding", "dem_oracle.c"),
    "dem_lubrication_radius": ("const double reff = ra * rb / (ra + rb);", "const double reff = 0.5 * (ra + rb);",
                               "test_oracle_dem.py", "lubrication", "dem_oracle.c"),
    "dem_wall_torque": ("cross3(arm, ft, t);", "cross3(ft, arm, t);", "test_oracle_dem.py", "sliding",
                        "dem_oracle.c"),
    "dem_inertia": ("D->inertia[i] = 0.4 * D->m[i] * r * r;", "D->inertia[i] = 0.5 * D->m[i] * r * r;",
                    "test_oracle_dem.py", "hydrodynamic", "dem_oracle.c"),
    "csf_corner_gradient": ("g[2] += st(phi, p * sx, q * sy, sz) - st(phi, p * sx, q * sy, 0);",
                            "g[2] += st(phi, p * sx, q * sy, sz) - st(phi, p * sx, q * sy, -sz);",
                            "test_oracle_geometry.py", "csf"),
    "csf_divergence_sign": ("div += 0.25 * (2 * c - 1) * nc[a][b][c][2];", "div -= 0.25 * (2 * c - 1) * nc[a][b][c][2];",
                            "test_oracle_geometry.py", "csf"),
    "csf_no_floor": ("-g[d] / (gn > CSF_GMIN ? gn : CSF_GMIN)", "-g[d] / (gn > 1e-12 ? gn : 1.0)",
                     "test_oracle_geometry.py", "continuous"),
    "dem_tangential_lubrication": ("(15.0 * (ra + rb) * (ra + rb) * (ra + rb))", "(10.0 * (ra + rb) * (ra + rb) * (ra + rb))",
                                   "test_oracle_dem.py", "tangential_lubrication_between", "dem_oracle.c"),
    "dem_tangential_lub_wall": ("8.0 * D->r[i] / 15.0", "8.0 * D->r[i] / 12.0",
                                "test_oracle_dem.py", "tangential_lubrication_against", "dem_oracle.c"),
    "galilean_sign": ("D1 -= 3.0 * (1.0 - 0.5 * omega) * (ex - ey);", "D1 += 3.0 * (1.0 - 0.5 * omega) * (ex - ey);",
                      "test_oracle_galilean.py", "sound_wave"),
    "galilean_source_factor": ("T -= 3.0 * (1.0 - 0.5 * omega_bulk) * (ex + ey + ez);",
                               "T -= 3.0 * (1.0 - omega_bulk) * (ex + ey + ez);",
                               "test_oracle_galilean.py", "sound_wave"),
    "galilean_dropped_term": ("D2 -= 3.0 * (1.0 - 0.5 * omega) * (ex - ez);", "D2 -= 3.0 * (1.0 - 0.5 * omega) * (ex);",
                              "test_oracle_galilean.py", "sound_wave or cube"),
    "galilean_strain_rate": ("- 0.5 * omega_bulk * trace_neq;\n        const double dyv",
                             "- 0.5 * omega * trace_neq;\n        const double dyv",
                             "test_oracle_galilean.py", "sound_wave or cube"),
    "estimator_angle_threshold": ("else if (angle > 30.0) rule = 3;", "else if (angle > 45.0) rule = 3;",
                                  "test_oracle_estimator.py", "bias_network", "mlp_oracle.c"),
    "estimator_length_range": ("else if (rn < 0.5 || rn > 2.0) rule = 2;", "else if (rn < 0.5 || rn > 3.0) rule = 2;",
                               "test_oracle_estimator.py", "bias_network", "mlp_oracle.c"),
    "estimator_kappa_weight": ("const double kap = kfd + 0.25 * y[3];", "const double kap = kfd + y[3];",
                               "test_oracle_estimator.py", "bias_network", "mlp_oracle.c"),
    "estimator_input_centre": ("x[k] = phi[k] - 0.5;", "x[k] = phi[k];",
                               "test_oracle_estimator.py", "single_path", "mlp_oracle.c"),
    "estimator_rule_order": ("if (solid_nb) rule = 1;\n    else if (rn < 0.5 || rn > 2.0) rule = 2;",
                             "if (rn < 0.5 || rn > 2.0) rule = 2;\n    else if (solid_nb) rule = 1;",
                             "test_oracle_estimator.py", "solid_neighbour", "mlp_oracle.c"),
    "estimator_solid_cells": ("if (y < 0 || L->type[y] == OL_SOLID) solid_nb = 1;", "if (y < 0) solid_nb = 1;",
                              "test_oracle_estimator.py", "lattice"),
    "curvature_sign": ("*kappa = -(tr - gHg) / (2.0 * gn);", "*kappa = (tr - gHg) / (2.0 * gn);",
                       "test_oracle_geometry.py", "quadratic or sphere"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new, target, sel = MUTANTS[name][:4]
    mutated = MUTANTS[name][4] if len(MUTANTS[name]) > 4 else "fsl_oracle.c"
    mdir = tmp_path / "oracle"
    mdir.mkdir()
    for f in ("fsl_oracle.c", "fsl_oracle.h", "mlp_oracle.c", "dem_oracle.c"):
        src = open(os.path.join(ROOT, "oracle", f)).read()
        if f == mutated:
            assert src.count(old) >= 1, "mutation site not found: " + name
            src = src.replace(old, new, 1)
        (mdir / f).write_text(src)
    so = str(mdir / "liboracle.so")
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                    "-o", so, str(mdir / "fsl_oracle.c"), str(mdir / "mlp_oracle.c"),
                    str(mdir / "dem_oracle.c"), "-lm"],
                   check=True)
    env = dict(os.environ, FSL_ORACLE_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, target), "-k", sel],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert "failed" in r.stdout or "passed" in r.stdout, r.stdout[-2000:]  # some pin ran
    assert r.returncode == 1, "mutant %s survived:\n%s" % (name, r.stdout[-2000:])
