"""Mutation check of the two-dimensional oracle's pins: each case plants one
plausible mistake in a copy of oracle2d.c (the printed f(x+i, y+i) typo,
zero padding, a wrong divisor, rounding instead of the floor, overlapping or misplaced quadrants, a dropped
cross term, a wrong sign or normalisation, a transposed 2D histogram, an
off-by-one in the prefix sums, the last-pair tie rule), builds it with the
unchanged oracle.c, and requires at least one pin to reject it."""
import os
import subprocess
import sys
import textwrap

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "mean_index_typo": ("int32_t yy = y + dy, xx = x + dx;", "int32_t yy = y + dy, xx = x + dy;"),
    "mean_divisor": ("g[(int64_t)y * W + x] = (int32_t)(sum / 9);", "g[(int64_t)y * W + x] = (int32_t)(sum / 8);"),
    "zero_padding": ("if (yy < 0)\n                        yy = 0;", "if (yy < 0)\n                        continue;"),
    "hist_transposed": ("h[(int64_t)f[i] * L + g[i]] += 1u;", "h[(int64_t)g[i] * L + f[i]] += 1u;"),
    "class2_overlaps": ("H2 = region_tsallis_direct(h, L, N, t + 1, L - 1, s + 1, L - 1, q, &w2);",
                        "H2 = region_tsallis_direct(h, L, N, t, L - 1, s, L - 1, q, &w2);"),
    "class2_wrong_quadrant": ("H2 = region_tsallis_direct(h, L, N, t + 1, L - 1, s + 1, L - 1, q, &w2);",
                              "H2 = region_tsallis_direct(h, L, N, t + 1, L - 1, 0, s, q, &w2);"),
    "drop_cross_term": ("return H1 + H2 + (1.0 - q) * H1 * H2;", "return H1 + H2;"),
    "entropy_sign": ("    return (1.0 - s) / (q - 1.0);\n}", "    return (1.0 - s) / (1.0 - q);\n}"),
    "no_normalisation": ("s += pow(p / w, q);", "s += pow(p, q);"),
    "prefix_suffix_offset": ("H2 = region_tsallis_prefix(z->CB[(int64_t)(t + 1) * L + s + 1], z->QB[(int64_t)(t + 1) * L + s + 1], N, q,",
                             "H2 = region_tsallis_prefix(z->CB[(int64_t)t * L + s], z->QB[(int64_t)t * L + s], N, q,"),
    "prefix_row_reset": ("            s += hij ? pow((double)hij / z->N, q) : 0.0;\n            z->CA",
                         "            s = hij ? pow((double)hij / z->N, q) : 0.0;\n            z->CA"),
    "tie_rule_last": ("if (!found || S > best) {", "if (!found || S >= best) {"),
    "mean_rounded": ("g[(int64_t)y * W + x] = (int32_t)(sum / 9);", "g[(int64_t)y * W + x] = (int32_t)((sum + 4) / 9);"),
}

RUNNER = textwrap.dedent("""
    import sys, warnings
    warnings.simplefilter("ignore")
    sys.path[:0] = [{root!r}, {tests!r}]
    import oracle, pins2d
    lib = oracle.load_library({lib!r})
    failed = []
    for pin in pins2d.ALL_PINS:
        try:
            pin(lib=lib)
        except Exception as e:
            failed.append(pin.__name__)
    print("FAILED:" + ",".join(failed))
""")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(os.path.join(ROOT, "oracle", "oracle2d.c")).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    c = tmp_path / "mutant2d.c"
    c.write_text(src.replace(old, new))
    so = str(tmp_path / "libmutant.so")
    oracle.compile_source([os.path.join(ROOT, "oracle", "oracle.c"), str(c)], so)
    code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=so)
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    if p.returncode != 0:  # a crash of the mutant also counts as caught
        return
    line = [x for x in p.stdout.splitlines() if x.startswith("FAILED:")][-1]
    failed = [x for x in line[len("FAILED:"):].split(",") if x]
    assert failed, f"no pin rejects mutant {name}"
