"""Planted mistakes: each mutation of the oracle's C source must be caught by
at least one of the pins in test_oracle_pins.py or test_oracle_next.py.  The mutant is compiled from
a patched copy of oracle/adop_oracle.c into a temporary directory and loaded
in place of the real oracle for the duration of one check (CPU only)."""
import os
import subprocess

import pytest

import tests.test_oracle_envmap as envpins
import tests.test_oracle_next as nxt
import tests.test_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "adop_oracle.c")

MICRO = {s["name"]: s for s in pins.MICRO}
TOL = {t["name"]: t for t in pins.TOL_SCALE}

# (id, original text, mutated text, check that must fail)
MUTANTS = [
    ("shift_sign", "double du = 0.5 * (right - left);", "double du = 0.5 * (right + left);",
     lambda O: pins.test_microscenes(O, MICRO["S1_empty_neighbours"])),
    ("layer_chain", "gu += ldexp(du, -l);", "gu += du;",
     lambda O: pins.test_microscenes(O, MICRO["S6_two_layers"])),
    ("case2_no_fuzz", "if (Z > behind) return 0.0;", "if (Z > minz) return 0.0;",
     lambda O: pins.test_spatial_gradient_equals_rerender(O, 21, 1)),
    ("case4_mean", "double Inew = ((double)nq * I + tau[ch]) / (double)(nq + 1);",
     "double Inew = ((double)nq * I + tau[ch]) / (double)(nq);",
     lambda O: pins.test_microscenes(O, MICRO["S4b_equal_depth_n3"])),
    ("case1_background", "double dI = tau[ch] - b;",
     "double dI = tau[ch];",
     lambda O: pins.test_microscenes(O, MICRO["S8_background"])),
    ("bg_image_ignored", "if (k == 0) return bg_image ? bg_image[o] : (double)background[ch];",
     "if (k == 0) return (double)background[ch];",
     lambda O: envpins.test_empty_pixels_take_the_per_pixel_background(O)),
    ("bg_image_case1_ignored", "double b = bg_image ? bg_image[o] : (double)background[ch];",
     "double b = (double)background[ch];",
     lambda O: envpins.test_empty_neighbour_uses_the_map_value(O)),
    ("dfeat_count", "dfeat[i * c + ch] += g / k * chain;", "dfeat[i * c + ch] += g * chain;",
     lambda O: pins.test_feature_gradient_finite_difference(O)),
    ("visible_gate", "if (!visible && !(flags & ORACLE_SPATIAL_ALL)) continue;",
     "if (0) continue;",
     lambda O: pins.test_microscenes(O, MICRO["S7_hidden_point"])),
    ("dpos_transpose", "s += (double)Rf[3 * j + k] * gc[j];", "s += (double)Rf[3 * k + j] * gc[j];",
     lambda O: pins.test_chain_rule_finite_difference(O, "distorted")),
    ("omega_sign", "double cr[3] = { xc[1] * gc[2] - xc[2] * gc[1],",
     "double cr[3] = { xc[2] * gc[1] - xc[1] * gc[2],",
     lambda O: pins.test_chain_rule_finite_difference(O, "distorted")),
    ("dintr_k2", "au * r2, au * r4, au * r6,", "au * r2, au * r2, au * r6,",
     lambda O: pins.test_chain_rule_finite_difference(O, "distorted")),
    ("tangential_swap", "float xd = fmaf(a, D, fmaf(cam->p1 + cam->p1, ab, tx));",
     "float xd = fmaf(a, D, fmaf(cam->p2 + cam->p2, ab, tx));",
     lambda O: pins.test_projection_distortion_vs_float64(O, "strong_tangential")),
    ("round_half_up", "float fx = rintf(ldexpf(u0, -l));", "float fx = floorf(ldexpf(u0, -l) + 0.5f);",
     lambda O: pins.test_rounding_ties_and_bounds(O)),
    ("fuzzy_off", "const float fa = 1.0f + alpha;\n    st->total", "const float fa = 1.0f;\n    st->total",
     lambda O: pins.test_forward_matches_brute_force(O, 2, 0.05)),
    ("tie_index", "uint64_t key = ((uint64_t)f2u(Z) << 32) | (uint64_t)(uint32_t)i;",
     "uint64_t key = ((uint64_t)f2u(Z) << 32) | (uint64_t)(uint32_t)(n - 1 - i);",
     lambda O: pins.test_forward_matches_brute_force(O, 1, 0.01)),
    ("bounds_closed", "fx < (float)wl && fy >= 0.0f && fy < (float)hl", "fx <= (float)wl && fy >= 0.0f && fy <= (float)hl",
     lambda O: pins.test_rounding_ties_and_bounds(O)),
    ("cull_sign", "if (opt->flags & ORACLE_CULL_BACKFACE) return d < 0.0f;",
     "if (opt->flags & ORACLE_CULL_BACKFACE) return d > 0.0f;",
     lambda O: nxt.test_normal_culling_equals_rendering_the_kept_subset(O, "backface")),
    ("cull_normal_untransformed", "float m2 = fmaf(R[6], nv[0], fmaf(R[7], nv[1], R[8] * nv[2]));",
     "float m2 = nv[2];",
     lambda O: nxt.test_normal_culling_equals_rendering_the_kept_subset(O, "printed")),
    ("log_chain", "double chain = (flags & ORACLE_LOG_FEATURES) ? tau[ch] : 1.0;", "double chain = 1.0;",
     lambda O: nxt.test_log_features_gradient_finite_difference(O)),
    ("discard_layer_scale", "float lhs = ldexpf(s0, -l) * opt->gamma;", "float lhs = s0 * opt->gamma;",
     lambda O: nxt.test_discard_equals_rendering_each_layers_kept_subset(O)),
    ("discard_no_sqrt", "float rhs = sqrtf(1.0f - opt->beta[i]);", "float rhs = 1.0f - opt->beta[i];",
     lambda O: nxt.test_discard_equals_rendering_each_layers_kept_subset(O)),
    ("knn_third", "radius[i] = sqrtf(best[3]);", "radius[i] = sqrtf(best[2]);",
     lambda O: nxt.test_knn_radius_against_kdtree(O)),
    # the tolerance yardstick S: inflated or deflated magnitudes
    ("scale_gc_inflated",
     "(fabs(a) * ga_m + fabs(b) * gb_m) / fabs(Zd) };",
     "(fabs(a) * ga_m + fabs(b) * gb_m + ga_m) / fabs(Zd) };",
     lambda O: pins.test_tolerance_scale_microscenes(O, TOL["S1_empty_neighbours"])),
    ("scale_intr_inflated",
     "double di_m[9] = { gu_m * fabs(xd), gv_m * fabs(yd), gu_m, gv_m,",
     "double di_m[9] = { gu_m * (fabs(xd) + 1.0), gv_m * fabs(yd), gu_m, gv_m,",
     lambda O: pins.test_tolerance_scale_microscenes(O, TOL["S1_empty_neighbours"])),
    ("scale_omega_inflated",
     "double cr_m[3] = { fabs(xc[1]) * gc_m[2] + fabs(xc[2]) * gc_m[1],",
     "double cr_m[3] = { fabs(xc[1]) * gc_m[2] + fabs(xc[2]) * gc_m[1] + gc_m[0],",
     lambda O: pins.test_tolerance_scale_microscenes(O, TOL["S2_neighbour_in_front"])),
    ("scale_dfeat_no_count",
     "if (dfeat_abs) dfeat_abs[i * c + ch] += fabs(g) / k * chain;",
     "if (dfeat_abs) dfeat_abs[i * c + ch] += fabs(g) * chain;",
     lambda O: pins.test_tolerance_scale_microscenes(O, TOL["S4b_equal_depth_n3"])),
    ("scale_case4_undivided",
     "m += fabs(g) * (fabs(tau[ch]) + fabs(I)) / (double)(nq + 1);",
     "m += fabs(g) * (fabs(tau[ch]) + fabs(I));",
     lambda O: pins.test_tolerance_scale_microscenes(O, TOL["S4b_equal_depth_n3"])),
    ("scale_shift_deflated",
     "gu_m += ldexp(0.5 * (mr + ml), -l);",
     "gu_m += ldexp(0.25 * (mr + ml), -l);",
     lambda O: pins.test_tolerance_scale_bounds_every_entry(O, 0)),
]


@pytest.mark.parametrize("mid,orig,mut,check", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(oracle, tmp_path, mid, orig, mut, check):
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation site for {mid} not unique/found"
    d = tmp_path / mid
    d.mkdir()
    (d / "adop_oracle.h").write_text(open(os.path.join(ROOT, "oracle", "adop_oracle.h")).read())
    (d / "adop_oracle.c").write_text(src.replace(orig, mut))
    so = str(d / "libmutant.so")
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-msse2",
                    "-mfpmath=sse", "-o", so, str(d / "adop_oracle.c"), "-lm"], check=True)
    saved = oracle._LIB
    oracle._LIB = oracle.load(so)
    try:
        with pytest.raises(AssertionError):
            check(oracle)
    finally:
        oracle._LIB = saved
