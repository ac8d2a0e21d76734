"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake into a copy of the C oracle (on the CPU, in a
temporary directory), builds it, and checks that at least one pin that does
not depend on the oracle fails: the hand-derived golden encodings and
perceptron outputs, or the agreement of the two neighbour searches.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "veckm_oracle.c")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "closed_form_encodings.json")

MUTATIONS = {
    "phase_sign": ("im[j] += sin(th);", "im[j] -= sin(th);"),
    "xy_columns_swapped": ("A[3 * j + 0] * (double)dx + A[3 * j + 1] * (double)dy",
                           "A[3 * j + 1] * (double)dx + A[3 * j + 0] * (double)dy"),
    "dropped_time_term": ("+\n                A[3 * j + 2] * (double)dt;", ";"),
    "exclusive_spatial_bound": ("if (iabs64(dx) > rx || iabs64(dy) > ry) return 0;",
                                "if (iabs64(dx) >= rx || iabs64(dy) > ry) return 0;"),
    "no_temporal_bound": ("if (rt >= 0 && iabs64(dt) > rt) return 0;", ""),
    "self_excluded": ("if (!in_window(dx, dy, dt, rx, ry, rt)) continue;",
                      "if (!in_window(dx, dy, dt, rx, ry, rt) || k == q) continue;"),
    "wrong_normaliser": ("row[j] = c > 0 ? re[j] / (double)c : 0.0;",
                         "row[j] = c > 0 ? re[j] / (double)(c + 1) : 0.0;"),
    "re_im_interleaved": ("row[D + j] = c > 0 ? im[j] / (double)c : 0.0;",
                          "row[D + j] = c > 0 ? re[j] / (double)c : 0.0;"),
    "bucket_row_off_by_one": ("for (int64_t py = yq - ry; py <= yq + ry; ++py) {",
                              "for (int64_t py = yq - ry; py < yq + ry; ++py) {"),
    "mlp_no_relu": ("if (h < 0.0) h = 0.0;", ""),
    "mlp_w1_transposed": ("const double* w = W1 + (size_t)r * (size_t)in_dim;\n"
                          "      for (int32_t c = 0; c < in_dim; ++c) h += w[c] * xi[c];",
                          "for (int32_t c = 0; c < in_dim && c < hidden; ++c)\n"
                          "        h += W1[(size_t)c * (size_t)in_dim + r] * xi[c];"),
    "mlp_dropped_output_bias": ("out[2 * i + 1] = o1 + b2[1];", "out[2 * i + 1] = o1;"),
    "mlp_w2_rows_swapped": ("o0 += W2[r] * h;", "o0 += W2[hidden + r] * h;"),
}


def _pins_pass(lib) -> bool:
    with open(GOLDEN) as f:
        g = json.load(f)
    A = np.array([[math.pi / 2, 0.0, 0.0], [0.0, math.pi / 3, math.pi]])
    ev = np.array(g["events_xytp"], dtype=np.int32)
    ok = True
    for search in ("scan", "bucket"):
        c0 = g["cases"][0]
        emb, cnt = oracle.encode(ev, A, *c0["radii"], search=search, lib=lib)
        ok &= np.array_equal(cnt, c0["cnt"])
        ok &= np.allclose(emb, c0["emb_planar"], atol=1e-12, rtol=0)
        c1 = g["cases"][1]
        emb1, cnt1 = oracle.encode(ev, A, *c1["radii"], queries=[c1["query"]], search=search,
                                   lib=lib)
        ok &= cnt1[0] == c1["cnt"]
        ok &= np.allclose(emb1[0], c1["emb_planar"], atol=1e-12, rtol=0)
    m = g["mlp"]
    x = np.array(g["cases"][0]["emb_planar"])[m["inputs_from_queries"]]
    out = oracle.mlp(x, m["W1"], m["b1"], m["W2"], m["b2"], lib=lib)
    ok &= np.allclose(out, m["flow"], atol=1e-12, rtol=0)
    rng = np.random.Generator(np.random.PCG64(5))
    ev2 = np.stack([rng.integers(0, 30, 600), rng.integers(0, 25, 600),
                    rng.integers(0, 8, 600), rng.choice([-1, 1], 600)], 1).astype(np.int32)
    A2 = rng.normal(size=(6, 3))
    e_scan, c_scan = oracle.encode(ev2, A2, 2, 3, 1, search="scan", lib=lib)
    e_buck, c_buck = oracle.encode(ev2, A2, 2, 3, 1, search="bucket", lib=lib)
    ok &= np.array_equal(c_scan, c_buck) and np.array_equal(e_scan, e_buck)
    return bool(ok)


def test_unmutated_oracle_passes_pins(tmp_path):
    lib = oracle.load_library(oracle.compile_source(SRC, str(tmp_path / "lib_clean.so")))
    assert _pins_pass(lib)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found: " + name
    mutated = tmp_path / ("oracle_%s.c" % name)
    mutated.write_text(src.replace(old, new))
    lib = oracle.load_library(oracle.compile_source(str(mutated), str(tmp_path / ("lib_%s.so" % name))))
    assert not _pins_pass(lib), "planted mistake '%s' was not caught" % name
