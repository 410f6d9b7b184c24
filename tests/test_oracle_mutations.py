"""The oracle pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle source (on the CPU),
builds it, points the oracle shim at the mutated build and runs the pin suite:
the suite must fail.  A mutation that survives means the pins do not
constrain that part of the oracle.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hj_oracle.c")

MUTATIONS = {
    "upwind_directions_swapped": ("*pm = (vc - vm) * inv_dx;\n        *pp = (vp - vc) * inv_dx;",
                                  "*pm = (vp - vc) * inv_dx;\n        *pp = (vc - vm) * inv_dx;"),
    "eno2_right_correction_sign": ("*pp = d1[2] - dx * eno_pick", "*pp = d1[2] + dx * eno_pick"),
    "eno2_picks_larger": ("return fabs(a) <= fabs(b) ? a : b;", "return fabs(a) <= fabs(b) ? b : a;"),
    "eno2_second_difference_scale": ("k < 3; ++k) d2[k] = (d1[k + 1] - d1[k]) * g->inv_2dx[d]",
                                     "k < 3; ++k) d2[k] = (d1[k + 1] - d1[k]) * inv_dx"),
    "weno_linear_weights_swapped": ("double a1 = 0.1 * r1, a2 = 0.6 * r2, a3 = 0.3 * r3;",
                                    "double a1 = 0.3 * r1, a2 = 0.6 * r2, a3 = 0.1 * r3;"),
    "weno_candidate_coefficient": ("v3 * C11_6", "v3 * C5_6"),
    "weno_smoothness_term": ("double fb = w[1] - w[3];", "double fb = w[1] + w[3];"),
    "weno_right_weights_order": ("w[4], w[3], w[2], w[1], w[0], r.rc, r.rb, r.ra",
                                 "w[4], w[3], w[2], w[1], w[0], r.ra, r.rb, r.rc"),
    "weno_right_stencil_order": ("*pp = weno_right(&d1[1]);", "*pp = weno_left(&d1[1]);"),
    "weno_eps_scale": ("double eps = 1e-6 * mx + 1e-99;", "double eps = 1e-4 * mx + 1e-99;"),
    "dubins4d_accel_sign": ("+ wm * fabs(p[2]) + am * fabs(p[3]);",
                            "+ wm * fabs(p[2]) - am * fabs(p[3]);"),
    "dubins4d_heading_swapped": ("return -p[0] * (v * g->cs[2][k]) - p[1] * (v * g->sn[2][k])",
                                 "return -p[0] * (v * g->sn[2][k]) - p[1] * (v * g->cs[2][k])"),
    "double_integrator_control_sign": ("return -p[0] * x2 + dy->prm[0] * fabs(p[1]);",
                                       "return -p[0] * x2 - dy->prm[0] * fabs(p[1]);"),
    "translation_sign": ("for (int d = 0; d < g->nd; ++d) h -= dy->prm[d] * p[d];",
                         "for (int d = 0; d < g->nd; ++d) h += dy->prm[d] * p[d];"),
    "lf_dissipation_sign": ("diss += a * ((pp[d] - pm[d]) / 2.0);",
                            "diss -= a * ((pp[d] - pm[d]) / 2.0);"),
    "rhs_sign": ("    return -hhat;\n}", "    return hhat;\n}"),
    "rk2_combination": ("v[k] = (v[k] + v2) / 2.0;", "v[k] = v2;"),
    "rk3_middle_stage": ("w2[k] = (3.0 * v[k] + v2) / 4.0;", "w2[k] = (v[k] + v2) / 2.0;"),
    "rk3_last_stage": ("v[k] = (v[k] + 2.0 * v3) / 3.0;", "v[k] = (2.0 * v[k] + v3) / 3.0;"),
    "tube_uses_max": ("if (v0[k] < v[k]) v[k] = v0[k];", "if (v0[k] > v[k]) v[k] = v0[k];"),
    "ghost_extrapolation_sign": ("return v0 + (double)(-j) * (v0 - v1);",
                                 "return v0 - (double)(-j) * (v0 - v1);"),
    "periodic_wrap_offset": ("long jj = ((j % n) + n) % n;", "long jj = ((j % n) + n + 1) % n;"),
    "rel_dubins_rotation_sign": ("fabs(p[0] * y - p[1] * x - p[2])", "fabs(p[0] * y + p[1] * x - p[2])"),
    "rel_dubins_pursuer_sign": ("+ wp * fabs(p[2]);", "- wp * fabs(p[2]);"),
    "rel_dubins_drift_sign": ("-p[0] * (-ve + vp * c)", "-p[0] * (ve + vp * c)"),
    "dubins4d_turn_sign": ("+ wm * fabs(p[2])", "- wm * fabs(p[2])"),
    "double_integrator_drift_sign": ("return -p[0] * x2 +", "return p[0] * x2 +"),
    "alpha_double_integrator": ("if (d == 0) return fabs(g->x[1][axis_index(g, node, 1)]);",
                                "if (d == 0) return dy->prm[0];"),
    "cfl_rate": ("rate += alpha[d] / g->dx[d];", "rate += alpha[d] * g->dx[d];"),
    "periodic_cell_size": ("(hi[d] - lo[d]) / (double)n[d]", "(hi[d] - lo[d]) / (double)(n[d] - 1)"),
    "rockets_evader_abs_argument": ("- um * fabs(p[0] * x - p[2])", "- um * fabs(p[0] * x + p[2])"),
    "rockets_pursuer_sign": ("+ um * fabs(p[1] * x + p[2]);", "- um * fabs(p[1] * x + p[2]);"),
    "rockets_gravity_sign": ("double drift2 = a * g->sn[2][k] + a - grav;",
                             "double drift2 = a * g->sn[2][k] + a + grav;"),
    "rockets_alpha_misses_x": ("if (d == 0) return fabs(a * g->cs[2][k]) + um * fabs(x);",
                               "if (d == 0) return fabs(a * g->cs[2][k]);"),
    "vi_restricts_the_wrong_way": ("if (mode == ORC_TUBE_VI && l > 0.0) l = 0.0;",
                                   "if (mode == ORC_TUBE_VI && l < 0.0) l = 0.0;"),
    "vi_restricts_nothing": ("if (mode == ORC_TUBE_VI && l > 0.0) l = 0.0;", ""),
    "tube_out_every_step": ("const int step_mode = mode == ORC_TUBE_OUT ? ORC_SET : mode;",
                            "const int step_mode = mode == ORC_TUBE_OUT ? ORC_TUBE : mode;"),
    "eno3_minus_factor_swapped": ("            cs = eno_pick(d3[0], d3[1]);\n            f = 2.0;",
                                  "            cs = eno_pick(d3[0], d3[1]);\n            f = -1.0;"),
    "eno3_picks_larger_third": ("            c = d2[3];\n            cs = eno_pick(d3[2], d3[3]);",
                                "            c = d2[3];\n            cs = eno_pick(d3[3], d3[2]) == d3[3] ? d3[2] : d3[3];"),
    "eno3_third_difference_scale": ("d3[k] = (d2[k + 1] - d2[k]) * g->inv_3dx[d];",
                                    "d3[k] = (d2[k + 1] - d2[k]) * g->inv_2dx[d];"),
    "eno3_right_first_difference": ("*pp = (d1[3] - c * dx) + cs * (f * dxx);",
                                    "*pp = (d1[2] - c * dx) + cs * (f * dxx);"),
    "box_sign_minus_never": ("    if (smin <= 0.0) {\n        double v = fabs(base - k);",
                             "    if (smin < -1e300) {\n        double v = fabs(base - k);"),
    "box_interval_ends_swapped": ("l = l + (u < w ? u : w);", "l = l + (u < w ? w : u);"),
    "glf_box_misses_right_derivative": ("            if (pp < lo) lo = pp;\n", ""),
    "llf_box_upper_from_left_only": ("hi[d] = pm[d] < pp[d] ? pp[d] : pm[d];", "hi[d] = pm[d];"),
    "rockets_box_p3_sign": ("double v = sign_max(-um, um, l2, h2);",
                            "double v = sign_max(-um, -um, l2, h2);"),
    "box_inside_term_dropped": ("return sqrt(outside) + (inside < 0.0 ? inside : 0.0);",
                                "return sqrt(outside);"),
    "ellipsoid_weight_outside_square": ("acc = acc + size[d] * (t * t);",
                                        "acc = acc + (size[d] * t) * (size[d] * t);"),
    "sphere_ignores_center": ("        double t = x[d] - c[d];\n", "        double t = x[d];\n"),
    "union_takes_max": ("v = sv < v ? sv : v;", "v = sv > v ? sv : v;"),
    "subtract_sign": ("v = -sv > v ? -sv : v;", "v = sv > v ? sv : v;"),
}

PIN_FILES = ("test_oracle_pins.py", "test_oracle_rockets_tubes.py", "test_oracle_shapes.py",
             "test_oracle_dissipation.py", "test_oracle_exact_derivs.py",
             "test_oracle_hamiltonians.py")

# The pin file that targets each group of mutations runs first (every pin
# file still runs until one test fails, so this only saves time).
FIRST_FILE = (("box_", "test_oracle_dissipation.py"), ("glf_", "test_oracle_dissipation.py"),
              ("llf_", "test_oracle_dissipation.py"),
              ("rockets_box", "test_oracle_dissipation.py"),
              ("rockets_", "test_oracle_rockets_tubes.py"), ("vi_", "test_oracle_rockets_tubes.py"),
              ("tube_out", "test_oracle_rockets_tubes.py"),
              ("ellipsoid", "test_oracle_shapes.py"), ("sphere", "test_oracle_shapes.py"),
              ("union", "test_oracle_shapes.py"), ("subtract", "test_oracle_shapes.py"),
              ("weno_", "test_oracle_exact_derivs.py"), ("eno", "test_oracle_exact_derivs.py"),
              ("upwind_", "test_oracle_exact_derivs.py"))


def _pin_order(name):
    first = next((f for pre, f in FIRST_FILE if name.startswith(pre)), PIN_FILES[0])
    return (first,) + tuple(f for f in PIN_FILES if f != first)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found: " + name
    mut = tmp_path / "hj_oracle_mut.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libhj_oracle_mut.so"
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-std=c99", "-o", str(lib), str(mut), "-lm"], check=True)
    env = dict(os.environ, HJ_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] +
                       [os.path.join(ROOT, "tests", f) for f in _pin_order(name)],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "mutation %s survived the pins:\n%s" % (name, r.stdout[-2000:])
