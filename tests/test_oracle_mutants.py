"""The oracle's pins detect plausible mistakes (CPU only).

Each case plants one mistake in a copy of the oracle's C source (a dropped
term, a wrong sign, a wrong index, a transposed operand ...), builds it, and
runs the pin suite against the mutant through FWRS_ORACLE_LIB.  The suite must
fail for every mutant.  The product library is not involved.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

from oracle import build as oracle_build  # noqa: E402

MUTANTS = {
    "philox_hi_lo_swapped": ("uint32_t y1 = lo_b;", "uint32_t y1 = hi_b;"),
    "philox_key_not_bumped": ("k1 += PHILOX_WEYL_B;", "k1 += 0u;"),
    "exp2_sign_of_f": ("p = p * f;", "p = p * -f;"),
    "density_drops_r_m_term": ("*den = T * t1;", "*den = T;"),
    "density_exponent_sign": ("-(e * o->C)", "(e * o->C)"),
    "weight_fovea_test_inverted": ("if (level == 0 || e <= o->rf) return 1.0f;",
                                   "if (level == 0 || e >= o->rf) return 1.0f;"),
    "weight_level_ignored": ("if (level == 0 || e <= o->rf)", "if (e <= o->rf)"),
    "bias_survival_not_complemented": ("float survive = 1.0f - q;", "float survive = q;"),
    "bias_dropped": ("W1b = W1 * survive;", "W1b = W1 * 1.0f;"),
    "combine_direction": ("if (u * s > W1b) {", "if (u * s < W1b) {"),
    "index_off_by_one": ("idx[(size_t)j * n] = t;", "idx[(size_t)j * n] = t + 1u;"),
    "slots_share_one_word": ("words[j % 4] >> 8", "words[0] >> 8"),
    "counter_pixel_frame_swapped": ("uint32_t ctr[4] = {p, t, (uint32_t)b, 0u};",
                                    "uint32_t ctr[4] = {t, p, (uint32_t)b, 0u};"),
    "uniform_not_offset": ("((words[j % 4] >> 8) + 1u)", "((words[j % 4] >> 8) + 0u)"),
    "stored_wsum_unbiased": ("*wsum = s;", "*wsum = W1 + w;"),
    "count_not_incremented": ("*cnt = *cnt + 1u;", "*cnt = *cnt;"),
    "colour_channels_mixed": ("col[((size_t)j * 3 + 1) * n] = rgb[1];", "col[((size_t)j * 3 + 1) * n] = rgb[0];"),
    "stored_weight_is_wsum": ("            wt[(size_t)j * n] = w;\n            idx[(size_t)j * n] = t;\n        }\n    }",
                              "            wt[(size_t)j * n] = s;\n            idx[(size_t)j * n] = t;\n        }\n    }"),
    "resolve_unnormalised": ("out[3 * p + c] = acc / total;", "out[3 * p + c] = acc;"),
    "resolve_wrong_slot_weight": ("acc += (double)o->wt[(size_t)j * n + p] *", "acc += (double)o->wt[p] *"),
    "eq7_colour_factor_dropped": ("float W1b = (W1 * (1.0f - dl)) * survive;", "float W1b = W1 * survive;"),
    "eq7_not_clamped": ("return fminf(1.0f, fwrs_oracle_de94(a, b) / 100.0f);",
                        "return fwrs_oracle_de94(a, b) / 100.0f;"),
    "lab_lightness_offset": ("lab[0] = 116.0f * fy - 16.0f;", "lab[0] = 116.0f * fy - 15.0f;"),
    "lab_knee_ignored": ("if (t > eps) return fwrs_oracle_cbrt(t);", "if (t > -1.0f) return fwrs_oracle_cbrt(t);"),
    "cie94_chroma_of_wrong_colour": ("float SC = 1.0f + 0.045f * C1;", "float SC = 1.0f + 0.045f * C2;"),
    "cbrt_midpoint_is_lower_neighbour": ("const u128 m = 2 * M + 1;", "const u128 m = 2 * M - 1;"),
    "cbrt_midpoint_exponent": ("return compare_scaled(m * m * m, 3 * (E - 1), T, Et);",
                               "return compare_scaled(m * m * m, 3 * E - 1, T, Et);"),
    "cbrt_single_precision_start": ("float y = (float)cbrt((double)t);", "float y = cbrtf(t) * (1.0f + 0x1p-22f);"),
    "xyz_matrix_entry": ("0.3575761f * g", "0.3757561f * g"),
    "reproject_motion_sign": ("const float sx = ((float)x + 0.5f) - motion[2 * p + 0];",
                              "const float sx = ((float)x + 0.5f) + motion[2 * p + 0];"),
    "reproject_rounds_to_nearest": ("const int qx = (int)floorf(sx);", "const int qx = (int)floorf(sx + 0.5f);"),
    "reproject_axes_swapped": ("q = (size_t)qy * (size_t)W + (size_t)qx;", "q = (size_t)qx * (size_t)W + (size_t)qy;"),
    "depth_test_absolute": ("if (fabsf(dc - dp) <= depth_tol * dc) keep = 1;", "if (fabsf(dc - dp) <= depth_tol) keep = 1;"),
    "depth_test_strict": ("if (fabsf(dc - dp) <= depth_tol * dc) keep = 1;",
                          "if (fabsf(dc - dp) < depth_tol * dc) keep = 1;"),
    "flush_keeps_count": ("                cnt[p] = 0u;\n", "                cnt[p] = o->cnt[p];\n"),
    "flush_keeps_wsum": ("                wsum[p] = 0.0f;\n", "                wsum[p] = o->wsum[p];\n"),
    "history_from_own_pixel": ("wsum[p] = o->wsum[q];", "wsum[p] = o->wsum[p];"),
    "depth_not_stored": ("dnew[p] = depth[p];", "dnew[p] = o->depth[p];"),
    "aes_key_times_weight": ("float kn = fwrs_oracle_log2u(words[j % 4]) / w;",
                             "float kn = fwrs_oracle_log2u(words[j % 4]) * w;"),
    "aes_empty_key_zero": ("return o->prm.bias_mode == FWRS_ORACLE_AES ? -INFINITY : 0.0f;",
                           "return o->prm.bias_mode == FWRS_ORACLE_AES ? 0.0f : 0.0f;"),
    "log2_variate_offset": ("const uint32_t m = (bits >> 8) + 1u;                 /* 1 .. 2^24 */",
                            "const uint32_t m = (bits >> 8) + 0u;                 /* 1 .. 2^24 */"),
    "log2_scale": ("log2l((long double)m) - 24.0L;", "log2l((long double)m) - 23.0L;"),
    "log2_truncated": ("    const float f = (float)v;\n", "    const float f = (float)(double)(float)(v * (1.0L - 0x1p-30L));\n"),
    "memoryless_decay_twice": ("W1b = W1 * o->decay;", "W1b = (W1 * o->decay) * o->decay;"),
    "mip_divisor_fixed": ("= s / (float)n;", "= s / 4.0f;"),
    "bilinear_no_half_texel": ("* inv_scale - 0.5f;", "* inv_scale;"),
    "bilinear_axes_mixed": ("const float top = t00 + fx * (t10 - t00);", "const float top = t00 + fy * (t10 - t00);"),
    "fovea_ring_not_squared": ("const float r0sq = r0 * r0, r1sq = r1 * r1;", "const float r0sq = r0, r1sq = r1 * r1;"),
    "gauss_sigma_not_squared": ("const float inv = 1.0f / (2.0f * sigma * sigma);", "const float inv = 1.0f / (2.0f * sigma);"),
    "gauss_unnormalised": ("for (int d = -R; d <= R; ++d) w[d + R] = w[d + R] / S;", "for (int d = -R; d <= R; ++d) w[d + R] = w[d + R];"),
    "blur_vertical_reads_source": ("acc = acc + w[d + R] * tmp[", "acc = acc + w[d + R] * src["),
    "gauss_levels_swapped": ("v = (lv == 1 ? a : b)", "v = (lv == 1 ? b : a)"),
    "decay_rate_not_natural": ("o->decay = fwrs_oracle_exp2p(-(p->lambda_decay * 1.44269504088896341f));",
                               "o->decay = fwrs_oracle_exp2p(-(p->lambda_decay));"),
}


def _run_mutant(name, tmpdir):
    old, new = MUTANTS[name]
    src = open(oracle_build.SRC).read()
    assert src.count(old) >= 1, f"{name}: pattern not found"   # every occurrence is mutated
    mpath = os.path.join(tmpdir, f"{name}.c")
    with open(mpath, "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(tmpdir, f"lib_{name}.so")
    hdr_dir = os.path.dirname(oracle_build.SRC)
    subprocess.run(["gcc", *oracle_build.CFLAGS, "-I", hdr_dir, "-o", lib, mpath, "-lm"], check=True,
                   capture_output=True)
    env = dict(os.environ, FWRS_ORACLE_LIB=lib, OMP_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_oracle_pins.py"), os.path.join(HERE, "test_oracle_eq7.py"),
                        os.path.join(HERE, "test_oracle_reproject.py"),
                        os.path.join(HERE, "test_oracle_ablations.py"),
                        os.path.join(HERE, "test_oracle_foveate.py")],
                       cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    return name, r.returncode, r.stdout[-400:]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    with cf.ThreadPoolExecutor(max_workers=6) as ex:
        results = list(ex.map(lambda n: _run_mutant(n, str(tmp_path)), sorted(MUTANTS)))
    survivors = [(n, out) for (n, rc, out) in results if rc == 0]
    assert not survivors, f"mutants not caught by any pin: {[n for n, _ in survivors]}"
