"""Planted-mistake check of the oracle pins (CPU only).

Each case copies the C oracle, plants one plausible mistake, builds it and
runs the pin suites (renderer and neural decode) against the mutated
library; the pins must fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "duplex_oracle.c")

MUTATIONS = {
    "weight_without_v": [("N[ch] += v * T * A[ch];", "N[ch] += T * A[ch];"),
                         ("D += v * T * B;", "D += T * B;")],
    "transmittance_without_v": [("P *= 1.0 - v * alpha;", "P *= 1.0 - alpha;")],
    "inner_sums_with_v_alpha": [("for (int ch = 0; ch < 3; ch++) A[ch] += alpha * G->col[ch];\n            B += alpha;",
                                 "for (int ch = 0; ch < 3; ch++) A[ch] += v * alpha * G->col[ch];\n            B += v * alpha;")],
    "power_missing_half": [("double pw = -0.5 * (G->con[0] * dx * dx + 2.0 * G->con[1] * dx * dy + G->con[2] * dy * dy);\n            double alpha = G->op * exp(pw);\n            if (alpha > c->o.amax) alpha = c->o.amax;\n            if (!decide_ge(st, alpha, c->o.amin, c->o.band_a)) continue;\n            for (int ch = 0; ch < 3; ch++) A",
                            "double pw = -(G->con[0] * dx * dx + 2.0 * G->con[1] * dx * dy + G->con[2] * dy * dy);\n            double alpha = G->op * exp(pw);\n            if (alpha > c->o.amax) alpha = c->o.amax;\n            if (!decide_ge(st, alpha, c->o.amin, c->o.band_a)) continue;\n            for (int ch = 0; ch < 3; ch++) A")],
    "cross_term_sign": [("o->con[1] = -b / det;", "o->con[1] = b / det;")],
    "no_dilation": [("double a = cov[0] + delta, b = cov[1], c = cov[2] + delta;",
                     "double a = cov[0], b = cov[1], c = cov[2];")],
    "transposed_view_in_jacobian": [("Mx[3 * a + j] = J[3 * a] * k->Rd[j] + J[3 * a + 1] * k->Rd[3 + j] + J[3 * a + 2] * k->Rd[6 + j];",
                                     "Mx[3 * a + j] = J[3 * a] * k->Rd[3 * j] + J[3 * a + 1] * k->Rd[3 * j + 1] + J[3 * a + 2] * k->Rd[3 * j + 2];")],
    "quaternion_sign": [("R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);",
                         "R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y + w * z);")],
    "fp32_view_transposed": [("o[i] = ((k->R[i * 3 + 0] * p[0] + k->R[i * 3 + 1] * p[1]) + k->R[i * 3 + 2] * p[2]) + k->t[i];",
                              "o[i] = ((k->R[0 * 3 + i] * p[0] + k->R[1 * 3 + i] * p[1]) + k->R[2 * 3 + i] * p[2]) + k->t[i];")],
    "sh_sign": [("Y[1] = -c1 * y;", "Y[1] = c1 * y;")],
    "sh_l3_constant": [("Y[12] = 0.25 * sqrt(7.0 / PI)", "Y[12] = 0.25 * sqrt(5.0 / PI)")],
    "sh_no_offset": [("double s = 0.5;", "double s = 0.0;")],
    "no_colour_clamp": [("o->col[ch] = s > 0 ? s : 0;", "o->col[ch] = s;")],
    "v_without_sigmoid": [("return 1.0 / (1.0 + exp(-s));", "return s;")],
    "depth_descending": [("if (x->depth != y->depth) return x->depth < y->depth ? -1 : 1;",
                          "if (x->depth != y->depth) return x->depth < y->depth ? 1 : -1;")],
    "tile_id_transposed": [("e[i].tile = (uint32_t)(ty * TX + tx);", "e[i].tile = (uint32_t)(tx * TY + ty);")],
    "no_aabb_gate": [("if (!c->gvis[g] || !in_rect(c->grect + 4 * g, px, py)) continue; /* AABB skip */",
                      "if (!c->gvis[g]) continue;")],
    "no_alpha_clamp": [("if (alpha > c->o.amax) alpha = c->o.amax;\n            if (!decide_ge(st, alpha, c->o.amin, c->o.band_a)) continue;\n            for (int ch = 0; ch < 3; ch++) A",
                        "if (!decide_ge(st, alpha, c->o.amin, c->o.band_a)) continue;\n            for (int ch = 0; ch < 3; ch++) A")],
    # 3DGS-style rule: drop the cell whose own product would push T below eps
    "et_excludes_crossing_cell": [("if (!no_et && !decide_ge(st, T, c->o.eps, c->o.band_T)) break; /* cell-level ET */", ""),
                                  ("        for (int ch = 0; ch < 3; ch++) N[ch] += v * T * A[ch];",
                                   "        if (!no_et && T * P < c->o.eps) break;\n        for (int ch = 0; ch < 3; ch++) N[ch] += v * T * A[ch];")],
    "no_cell_pad": [("float hx = kappa * sqrtf(cov[0]) + pad;", "float hx = kappa * sqrtf(cov[0]);")],
    "empty_pixel_not_bg": [("out->C[ch] = D > 0 ? N[ch] / D : c->o.bg[ch];", "out->C[ch] = D > 0 ? N[ch] / D : 0.0;")],
    # the LC-WSR cell weights of the "w/o T^cell" mode
    "lcwsr_no_depth_clamp": [("vv[n] *= lin > 0 ? lin : 0.0;", "vv[n] *= lin;")],
    "lcwsr_weight_grows_with_depth": [("double lin = 1.0 - cell_depth64(&k, n, cell_pos) / tau;",
                                       "double lin = cell_depth64(&k, n, cell_pos) / tau;")],
    "lcwsr_without_v": [("vv[n] *= lin > 0 ? lin : 0.0;", "vv[n] = lin > 0 ? lin : 0.0;")],
    "lcwsr_terminates": [("        int n = c->ids[i];\n        double w = c->v[n];",
                          "        if (D > 1.0) break;\n        int n = c->ids[i];\n        double w = c->v[n];")],
    # the termination-ratio counters (Sec. VII) and the last contributing entry
    "nval_with_termination": [("if (mode == 0) walk_duplex(&c, px, py, &sv, 1, &rv);",
                               "if (mode == 0) walk_duplex(&c, px, py, &sv, c.o.no_et, &rv);")],
    "nrend_counts_cells": [("if (cnt) { last = i - s + 1; nrend += cnt; }", "if (cnt) { last = i - s + 1; nrend += 1; }")],
    "last_requires_transmittance_drop": [("if (cnt) { last = i - s + 1; nrend += cnt; }",
                                          "if (cnt && P < 1.0) { last = i - s + 1; nrend += cnt; }")],
    # the neural decode
    "decode_no_relu": [("h[j] = acc > 0.0f ? acc : 0.0f;", "h[j] = acc;")],
    "decode_no_scale_clamp": [("r = r < lim ? r : lim;", "")],
    "decode_offset_not_rotated": [("means[3 * g + a] = p[a] + ((R[3 * a] * u[0] + R[3 * a + 1] * u[1]) + R[3 * a + 2] * u[2]);",
                                   "means[3 * g + a] = p[a] + u[a];")],
    "decode_inputs_swapped": [("x[F] = dist;\n            x[F + 1] = ex / dist;",
                               "x[F + 1] = dist;\n            x[F] = ex / dist;")],
    "decode_opacity_sigmoid": [("opac[g] = tanh((double)y[yoff[0] + kk]);",
                                "opac[g] = 1.0 / (1.0 + exp(-(double)y[yoff[0] + kk]));")],
    "decode_exp_short_series": [("    p = p * r + 1.0f / 120.0f;\n", "")],
    "decode_ratio_of_cell_scale_missing": [("scales[3 * g + a] = r * S[a];", "scales[3 * g + a] = r;")],
    "lcwsr_depth_along_x": [("return k->Rd[6] * pos[3 * n] + k->Rd[7] * pos[3 * n + 1] + k->Rd[8] * pos[3 * n + 2] + k->td[2];",
                             "return k->Rd[0] * pos[3 * n] + k->Rd[1] * pos[3 * n + 1] + k->Rd[2] * pos[3 * n + 2] + k->td[0];")],
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name, tmp_path):
    src = open(SRC).read()
    for old, new in MUTATIONS[name]:
        assert old in src, f"mutation anchor missing: {old[:60]}"
        src = src.replace(old, new, 1)
    cfile = tmp_path / "mut.c"
    cfile.write_text(src)
    lib = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                           "-o", str(lib), str(cfile), "-lm"])
    env = dict(os.environ, DUPLEX_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_decode_pins.py")], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"planted mistake '{name}' passed every pin"
