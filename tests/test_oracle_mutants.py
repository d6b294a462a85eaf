"""Planted mistakes in the oracle must be caught by its pins.

Each case copies ``oracle/gf_oracle.c``, makes one plausible slip in the copy
(a dropped term, a wrong sign, an off-by-one window, a swapped operand, a
wrong sampling index), builds it with gcc in a temporary directory, and runs
every pin against it: at least one pin has to fail.  The real oracle source
is never modified.  CPU only.
"""
import os

import pytest

import pins
from oracle import oracle

MUTANTS = {
    "count_off_by_one": ("(double)(y1 - y0 + 1) * (double)(x1 - x0 + 1)",
                         "(double)(y1 - y0 + 2) * (double)(x1 - x0 + 1)"),
    "window_too_narrow": ("k <= imin(w - 1, xx + r); ++k", "k <= imin(w - 1, xx + r - 1); ++k"),
    "row_window_unclipped_low": ("int y0 = imax(0, y - r), y1", "int y0 = imax(1, y - r), y1"),
    "variance_sign": ("corr_I[i] - mean_I[i] * mean_I[i]", "corr_I[i] + mean_I[i] * mean_I[i]"),
    "covariance_wrong_mean": ("corr_Ip[i] - mean_I[i] * mean_p[i]", "corr_Ip[i] - mean_I[i] * mean_I[i]"),
    "eps_halved": ("cov_Ip / (var_I + eps)", "cov_Ip / (var_I + 0.5 * eps)"),
    "b_sign": ("mean_p[i] - a[i] * mean_I[i]", "mean_p[i] + a[i] * mean_I[i]"),
    "corr_Ip_is_corr_I": ("tmp[i] = I[i] * p[i]", "tmp[i] = I[i] * I[i]"),
    "mean_b_from_a": ("oracle_box_mean_border(b, h, w, r, border, mb)", "oracle_box_mean_border(a, h, w, r, border, mb)"),
    "plain_output_swapped": ("qk[i] = ma[i] * I[i] + mb[i]", "qk[i] = mb[i] * I[i] + ma[i]"),
    "fast_uses_full_radius": ("coefficients(Il, pl, hl, wl, rl, eps, border, a, b)",
                              "coefficients(Il, pl, hl, wl, r, eps, border, a, b)"),
    "fast_skips_coefficient_mean": ("oracle_box_mean_border(a, hl, wl, rl, border, ma)",
                                    "oracle_box_mean_border(a, hl, wl, 0, border, ma)"),
    "lowres_radius_truncates": ("int rl = (2 * r + s) / (2 * s);", "int rl = r / s;"),
    "nearest_top_left": ("*t0 = imin(s * j + s / 2, n - 1);", "*t0 = imin(s * j, n - 1);"),
    "bilinear_centre": ("double u = (double)s * j + 0.5 * (double)(s - 1);",
                        "double u = (double)s * j + 0.5 * (double)s;"),
    "upsample_no_half_pixel": ("double u = ((double)y + 0.5) / (double)s - 0.5;",
                               "double u = (double)y / (double)s;"),
    "upsample_axes_swapped": ("(1.0 - wy) * ((1.0 - wx) * v00 + wx * v01) + wy * ((1.0 - wx) * v10 + wx * v11);\n        }\n    }\n    return 0;\n}\n\n/*\n * Algorithm 1",
                              "(1.0 - wx) * ((1.0 - wy) * v00 + wy * v01) + wx * ((1.0 - wy) * v10 + wy * v11);\n        }\n    }\n    return 0;\n}\n\n/*\n * Algorithm 1"),
    "upsample_wrong_tap": ("int ya = iclamp((int)fu, 0, hl - 1)", "int ya = iclamp((int)fu + 1, 0, hl - 1)"),
    "fast_output_uses_mean_b_twice": ("qk[i] = ua[i] * I[i] + ub[i]", "qk[i] = ub[i] * I[i] + ub[i]"),
    "joint_uses_full_radius": ("coefficients(Is, pc, hs, ws, rs, eps, border, ak, bk)",
                               "coefficients(Is, pc, hs, ws, r, eps, border, ak, bk)"),
    "joint_output_swapped": ("qc[i] = uak[i] * I[i] + ubk[i]", "qc[i] = ubk[i] * I[i] + uak[i]"),
    "joint_guide_wrong_mode": ("oracle_subsample(I, h, w, s, mode, Is)", "oracle_subsample(I, h, w, s, 1 - mode, Is)"),
    "joint_skips_b_mean": ("oracle_box_mean_border(bk, hs, ws, rs, border, mbk)",
                           "oracle_box_mean_border(bk, hs, ws, 0, border, mbk)"),
    "detail_sign": ("e[i] = q[i] + gain * (p[i] - q[i])", "e[i] = q[i] + gain * (q[i] - p[i])"),
    "detail_base_is_input": ("e[i] = q[i] + gain * (p[i] - q[i])", "e[i] = p[i] + gain * (p[i] - q[i])"),
    "reflect_repeats_low_edge": ("if (i < 0) i = -i;", "if (i < 0) i = -i - 1;"),
    "reflect_repeats_high_edge": ("if (i > n - 1) i = 2 * (n - 1) - i;", "if (i > n - 1) i = 2 * n - 1 - i;"),
    "replicate_wraps_around": ("if (border == ORACLE_REPLICATE) return iclamp(i, 0, n - 1);",
                               "if (border == ORACLE_REPLICATE) return (i % n + n) % n;"),
    "padded_count_short": ("const double count = (double)(2 * r + 1) * (double)(2 * r + 1);",
                           "const double count = (double)(2 * r + 1) * (double)(2 * r);"),
    "padded_row_window_short": ("for (int k = -r; k <= r; ++k) acc += x[", "for (int k = -r; k < r; ++k) acc += x["),
    "padded_column_reflects_rows_only": ("acc += rowsum[(size_t)border_index(y + k, h, border) * w + xx]",
                                         "acc += rowsum[(size_t)iclamp(y + k, 0, h - 1) * w + xx]"),
    "fast_ignores_border": ("if ((rc = coefficients(Il, pl, hl, wl, rl, eps, border, a, b))) goto done;",
                            "if ((rc = coefficients(Il, pl, hl, wl, rl, eps, ORACLE_CLIP, a, b))) goto done;"),
    "area_divides_by_full_block": ("acc / ((double)(y1 - y0) * (double)(x1 - x0))", "acc / ((double)s * (double)s)"),
    "area_block_shifted": ("int x0 = s * xx, x1 = imin(w, s * xx + s);", "int x0 = s * xx + s / 2, x1 = imin(w, s * xx + s);"),
    "color_eps_off_diagonal": ("M[3 * j + j] += eps;", "M[3 * j + ((j + 1) % 3)] += eps;"),
    "color_cov_wrong_mean": ("cov[j] = cIp[(size_t)j * n + i] - mI[(size_t)j * n + i] * mp[i];",
                             "cov[j] = cIp[(size_t)j * n + i] - mI[(size_t)j * n + i] * mI[(size_t)j * n + i];"),
    "color_adjugate_sign": ("adj[1] = M[2] * M[7] - M[1] * M[8];", "adj[1] = M[1] * M[8] - M[2] * M[7];"),
    "color_determinant_sign": ("double det = M[0] * adj[0] + M[1] * adj[3] + M[2] * adj[6];",
                               "double det = M[0] * adj[0] + M[1] * adj[3] - M[2] * adj[6];"),
    "color_b_one_channel_mean": ("bi -= x[j] * mI[(size_t)j * n + i];", "bi -= x[j] * mI[i];"),
    "color_cross_terms_dropped": ("for (size_t i = 0; i < n; ++i) tmp[i] = Ij[i] * Ik[i];",
                                  "for (size_t i = 0; i < n; ++i) tmp[i] = Ij[i] * Ij[i];"),
    "color_output_skips_plane": ("        for (int j = 0; j < 3; ++j) {\n            if ((rc = oracle_box_mean_border(ca + (size_t)j * nl, hl, wl, rl, border, mean_lo))) goto done;\n            if ((rc = oracle_upsample(mean_lo, hl, wl, s, h, w, up))) goto done;\n            const double *Ij",
                                 "        for (int j = 0; j < 2; ++j) {\n            if ((rc = oracle_box_mean_border(ca + (size_t)j * nl, hl, wl, rl, border, mean_lo))) goto done;\n            if ((rc = oracle_upsample(mean_lo, hl, wl, s, h, w, up))) goto done;\n            const double *Ij"),
    "color_joint_full_radius": ("if ((rc = coefficients_color(Il, p_lo + (size_t)k * nl, hl, wl, rl, eps, border, ca, cb))) goto done;",
                                "if ((rc = coefficients_color(Il, p_lo + (size_t)k * nl, hl, wl, r, eps, border, ca, cb))) goto done;"),
    "color_joint_guide_unsubsampled_plane": ("            for (size_t i = 0; i < n; ++i) qk[i] += up[i] * I[(size_t)j * n + i];",
                                             "            for (size_t i = 0; i < n; ++i) qk[i] += up[i] * I[i];"),
    "color_output_planes_swapped": ("const double *Ij = I + (size_t)j * n;\n            for (size_t i = 0; i < n; ++i) qk[i] += up[i] * Ij[i];",
                                    "const double *Ij = I + (size_t)(2 - j) * n;\n            for (size_t i = 0; i < n; ++i) qk[i] += up[i] * Ij[i];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    mpath = os.path.join(tmp_path, "mutant.c")
    with open(mpath, "w") as f:
        f.write(src.replace(old, new))
    lib = oracle.build(os.path.join(tmp_path, "libmutant.so"), mpath)
    orc = oracle.Oracle(lib)
    failed = []
    for pin in pins.ALL_PINS:
        try:
            pin(orc)
        except (AssertionError, RuntimeError, ValueError, FloatingPointError):
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"
