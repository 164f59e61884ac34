"""Mutation check of the morphology oracle's pins: each case plants one
plausible mistake in a copy of morph.c (a square instead of a disk, a disk
without its boundary, a cut row of the disk, zero padding at the border,
closing instead of opening, the subtraction reversed), builds it with the
unchanged oracle sources, and requires at least one pin to reject it."""
import os
import subprocess
import sys
import textwrap

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = {
    "square_element": ("if (dx * dx + dy * dy > r * r)", "if (0)"),
    "disk_without_boundary": ("if (dx * dx + dy * dy > r * r)", "if (dx * dx + dy * dy >= r * r)"),
    "disk_row_cut": ("for (int32_t dy = -r; dy <= r; ++dy)", "for (int32_t dy = -r; dy < r; ++dy)"),
    "zero_padding": ("continue; /* outside the image */",
                     "{ if (take_max ? 0 > best : 0 < best) best = 0; continue; }"),
    "closing_not_opening": ("or_morph(f, H, W, r, 0, tmp);\n    or_morph(tmp, H, W, r, 1, opened);",
                            "or_morph(f, H, W, r, 1, tmp);\n    or_morph(tmp, H, W, r, 0, opened);"),
    "residue_reversed": ("residue[i] = f[i] - opened[i];", "residue[i] = opened[i] - f[i];"),
}

RUNNER = textwrap.dedent("""
    import sys, warnings
    warnings.simplefilter("ignore")
    sys.path[:0] = [{root!r}, {tests!r}]
    import oracle, pins_morph
    lib = oracle.load_library({lib!r})
    failed = []
    for pin in pins_morph.ALL_PINS:
        try:
            pin(lib=lib)
        except Exception as e:
            failed.append(pin.__name__)
    print("FAILED:" + ",".join(failed))
""")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(os.path.join(ROOT, "oracle", "morph.c")).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    c = tmp_path / "mutant_morph.c"
    c.write_text(src.replace(old, new))
    so = str(tmp_path / "libmutant.so")
    oracle.compile_source([os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "oracle", "oracle2d.c"),
                           str(c)], so)
    code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=so)
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    if p.returncode != 0:  # a crash of the mutant also counts as caught
        return
    line = [x for x in p.stdout.splitlines() if x.startswith("FAILED:")][-1]
    failed = [x for x in line[len("FAILED:"):].split(",") if x]
    assert failed, f"no pin rejects mutant {name}"
