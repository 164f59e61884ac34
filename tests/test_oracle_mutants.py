"""Mutation check of the oracle's pins.

Each case plants one plausible mistake in a copy of oracle.c (a dropped term,
a wrong sign, index or bound, a transposed operand, a wrong tie rule), builds
it with gcc on the CPU and runs every pin against it in a child process.  The
case passes only if at least one pin rejects the mutant, i.e. the pins would
have caught that mistake in the oracle.
"""
import os
import subprocess
import sys
import textwrap

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "drop_cross_term": ("T = T + S[j] + (1.0 - q) * T * S[j];", "T = T + S[j];"),
    "cross_term_sign": ("T = T + S[j] + (1.0 - q) * T * S[j];", "T = T + S[j] + (q - 1.0) * T * S[j];"),
    "entropy_sign": ("return (1.0 - s) / (q - 1.0);", "return (1.0 - s) / (1.0 - q);"),
    "prefix_entropy_sign": ("return (1.0 - dq / pow(w, q)) / (q - 1.0);", "return (1.0 - dq / pow(w, q)) / (1.0 - q);"),
    "no_normalisation": ("s += pow(p[i] / w, q);", "s += pow(p[i], q);"),
    "prefix_no_normalisation": ("return (1.0 - dq / pow(w, q)) / (q - 1.0);", "return (1.0 - dq / w) / (q - 1.0);"),
    "transposed_pow": ("s += pow(p[i] / w, q);", "s += pow(q, p[i] / w);"),
    "class_overlap": ("        a = b + 1;\n    }\n    if (cx->comp", "        a = b;\n    }\n    if (cx->comp"),
    "threshold_range": ("        t[j] = j;\n    int found = 0;", "        t[j] = j + 1;\n    int found = 0;"),
    "tie_rule_last": ("if (!found || S > b1) {", "if (!found || S >= b1) {"),
    "argmin": ("if (!found || S > b1) {", "if (!found || S < b1) {"),
    "bin_width": ("int64_t W = (int64_t)hi - (int64_t)lo + 1;", "int64_t W = (int64_t)hi - (int64_t)lo;"),
    "clip_then_map": ("    if (v > hi)\n        return L - 1;\n", "    if (v > hi)\n        v = hi;\n"),
    "label_ge": ("if (b > thr[j])", "if (b >= thr[j])"),
    "prefix_mass_from_q": ("P[i] = (double)C / (double)N;", "P[i] = acc;"),
    "prefix_reset": ("acc += pow((double)hist[i] / (double)N, q);", "acc = pow((double)hist[i] / (double)N, q);"),
    "prefix_class_start": ("double dq = Q[b] - (a > 0 ? Q[a - 1] : 0.0);", "double dq = Q[b] - Q[a];"),
    "sumprod_drop_product": ("return kapur ? sum : sum + (1.0 - q) * prod;", "return sum;"),
    "sumprod_product_sign": ("return kapur ? sum : sum + (1.0 - q) * prod;", "return kapur ? sum : sum + (q - 1.0) * prod;"),
    "sumprod_product_skips_first": ("        prod *= S[j];\n", "        prod *= (j ? S[j] : 1.0);\n"),
    "sumprod_composes_recursively": ("    if (cx->comp == OR_COMP_SUMPROD)\n", "    if (0)\n"),
    "dp_sum_of_entropies": ("f[(int64_t)a * L + b] = isnan(S) ? -INFINITY : (kapur ? S : sgn * log(1.0 + (1.0 - q) * S));",
                            "f[(int64_t)a * L + b] = isnan(S) ? -INFINITY : S;"),
    "dp_short_range": ("for (int32_t t = a; t <= L - 1 - m; ++t) {", "for (int32_t t = a; t < L - 1 - m; ++t) {"),
    "dp_last_tuple": ("        int32_t t = a;\n        while (t <= L - 1 - m && !(f[(int64_t)a * L + t] + W[(size_t)(m - 1) * L + t + 1] == want))\n            ++t;",
                      "        int32_t t = L - 1 - m;\n        while (t > a && !(f[(int64_t)a * L + t] + W[(size_t)(m - 1) * L + t + 1] == want))\n            --t;"),
    "empty_class_allowed": ("    if (!(w > 0.0))\n        return NAN;\n    double s = 0.0;\n    for (int32_t i = a; i <= b; ++i)\n        if (p[i] > 0.0)\n            s += pow",
                            "    if (!(w > 0.0))\n        return 0.0;\n    double s = 0.0;\n    for (int32_t i = a; i <= b; ++i)\n        if (p[i] > 0.0)\n            s += pow"),
}

RUNNER = textwrap.dedent("""
    import sys, warnings
    warnings.simplefilter("ignore")
    sys.path[:0] = [{root!r}, {tests!r}]
    import oracle, pins
    lib = oracle.load_library({lib!r})
    failed = []
    for pin in pins.ALL_PINS:
        modes = [oracle.MODE_DIRECT, oracle.MODE_PREFIX] if pin in pins.MODE_PINS else [None]
        for m in modes:
            try:
                pin(lib=lib) if m is None else pin(lib=lib, mode=m)
            except Exception as e:
                failed.append(pin.__name__ + ("" if m is None else "[%d]" % m))
    print("FAILED:" + ",".join(failed))
""")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new)
    c = tmp_path / "mutant.c"
    c.write_text(mutated)
    so = str(tmp_path / "libmutant.so")
    oracle.compile_source(str(c), so)
    code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=so)
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    # a crash of the mutant also counts as caught, but report it
    if p.returncode != 0:
        assert p.returncode != 0, p.stderr
        return
    line = [x for x in p.stdout.splitlines() if x.startswith("FAILED:")][-1]
    failed = [x for x in line[len("FAILED:"):].split(",") if x]
    assert failed, f"no pin rejects mutant {name}"
