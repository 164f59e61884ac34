"""Host logic of bench.py that needs no GPU: the HBM-traffic record is used
only for the source and workload it was measured on, and the oracle's timed
sample is repeated until the minimum CPU time has run."""
import json
import os
import shutil

import numpy as np
import pytest

import bench
from paper_2012_10684_amd import synth


@pytest.fixture()
def tree(tmp_path, monkeypatch):
    """A copy of the kernel sources the record hashes and a traffic record
    for k_label.hip taken on them (workload volume300)."""
    src = os.path.join(bench.ROOT, "paper_2012_10684_amd", "csrc")
    dst = tmp_path / "paper_2012_10684_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in ("k_label.hip", "label_dev.h", "common.h", "morph_dev.h", "k_morph.hip"):
        shutil.copy(os.path.join(src, f), dst / f)
    (tmp_path / "include").mkdir()
    shutil.copy(os.path.join(bench.ROOT, "include", "ts.h"), tmp_path / "include" / "ts.h")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    rec = {"k_label.hip:volume300": {"src_sha": bench.src_hash("k_label.hip"), "workload": "volume300",
                                     "bytes_per_launch": 123.0},
           "k_label.hip:batch64": {"src_sha": "0" * 16, "workload": "batch64", "bytes_per_launch": 7.0},
           "k_morph.hip:volume300_open": {"src_sha": bench.src_hash("k_morph.hip"), "workload": "volume300_open",
                                          "bytes_per_launch": 5.0,
                                          "kernels": {"ts::k_morph<true, 10>(ts::MorphArgs)": 5.0,
                                                      "ts::k_morph<false, 10>(ts::MorphArgs)": 4.0}}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    return dst


def test_include_found_as_the_build_finds_it(tree):
    with open(tree / "k_label.hip", "a") as f:
        f.write('\n#include "ts.h"\n#include "hip/hip_runtime.h"\n')  # via -I include/; a system header
    files = bench.src_files("k_label.hip")
    assert os.path.join("..", "..", "include", "ts.h") in files
    assert not any("hip_runtime" in f for f in files)


def test_hash_covers_the_include_closure():
    files = bench.src_files("k_label.hip")
    assert files[0] == "k_label.hip"
    assert set(files[1:]) == {"label_dev.h", "common.h", os.path.join("..", "..", "include", "ts.h")}
    assert "morph_dev.h" not in bench.src_files("k_search.hip")


def test_traffic_used_for_its_source_and_workload(tree):
    assert bench.load_traffic("k_label.hip", "volume300") == 123.0
    assert bench.load_traffic("k_label.hip", "volume600") is None  # another workload
    assert bench.load_traffic("k_label.hip", "batch64") is None  # taken on another source
    assert bench.load_traffic("k_histogram.hip", "volume300") is None  # no record


@pytest.mark.parametrize("changed", ["k_label.hip", "label_dev.h", "common.h", "../../include/ts.h"])
def test_traffic_dropped_once_the_kernel_changes(tree, changed):
    with open(tree / changed, "a") as f:
        f.write("\nstatic const int edited = 1;\n")
    assert bench.load_traffic("k_label.hip", "volume300") is None


@pytest.mark.parametrize("edit", ["\n// a comment\n", "\n/* a\n   block */\n", "\n\n   \n"])
def test_traffic_kept_when_only_comments_or_blanks_change(tree, edit):
    with open(tree / "label_dev.h", "a") as f:
        f.write(edit)
    assert bench.load_traffic("k_label.hip", "volume300") == 123.0


def test_code_text_keeps_the_code():
    a = bench.code_text("int a = 1; // one\n/* two */ int b =  2;")
    assert a == "int a = 1; int b = 2;"
    assert bench.code_text("x = 1 - 2;") != bench.code_text("x = 1 + 2;")


def test_traffic_kept_when_a_header_it_does_not_include_changes(tree):
    with open(tree / "morph_dev.h", "a") as f:
        f.write("\nstatic const int edited = 1;\n")
    assert bench.load_traffic("k_label.hip", "volume300") == 123.0
    assert bench.load_traffic_sum("k_morph.hip", "volume300_open", ["ts::k_morph<false, 10>"]) is None


def test_traffic_sum_of_the_two_passes(tree):
    both = ["ts::k_morph<false, 10>", "ts::k_morph<true, 10>"]
    assert bench.load_traffic_sum("k_morph.hip", "volume300_open", both) == 9.0
    assert bench.load_traffic_sum("k_morph.hip", "volume300_open", ["ts::k_morph<true, 11>"]) is None  # no such kernel
    assert bench.load_traffic_sum("k_morph.hip", "volume300_open", ["ts::k_morph<"]) is None  # ambiguous prefix
    assert bench.load_traffic_sum("k_label.hip", "volume300", both) is None  # record without per-kernel bytes


def test_cpu_baseline_repeats_a_short_sample(monkeypatch):
    monkeypatch.setattr(bench, "CPU_MIN_S", 0.3)
    vol = synth.workload_slice(0)[None]
    base, check = bench.cpu_baseline([(0, vol[0])], bench.WORKLOADS["slice"], np.array([[[0]]]), np.array([[1.0]]),
                                     "one slice")
    for rec in (base, base["single_thread"]):
        passes = int(rec["sample"].split(" pass")[0].rsplit(" ", 1)[-1])
        assert passes >= 2, rec
        assert np.isfinite(rec["value"]) and rec["value"] > 0
    assert base["cores"] == 1 and base["single_thread"]["cores"] == 1  # one problem: one thread
    assert base["kind"] == "oracle" and base["cpu_model"]
    assert check["problems"] == 1  # the agreement check covers the sample once


def test_cpu_baseline_threads_take_whole_problems(monkeypatch):
    """Several problems: the multi-threaded timing uses up to the requested
    threads, and the agreement check compares every problem of the sample
    with the GPU's result at its own index."""
    import oracle
    monkeypatch.setattr(bench, "CPU_MIN_S", 0.2)
    wl = bench.WORKLOADS["batch64"]
    _, _, lo, hi, L, k, qs = wl
    vol = synth.make_volume(synth.rng_for(9, 3), 3, 128)
    sample = [(5, vol[0]), (2, vol[1]), (9, vol[2])]
    thr = np.full((1, 10, k), -1, np.int32)
    obj = np.full((1, 10), np.nan)
    for i, v in sample:
        r = oracle.search(oracle.histogram(v, lo, hi, L), k, qs[0])
        thr[0, i], obj[0, i] = r.thr, r.obj
    base, check = bench.cpu_baseline(sample, wl, thr, obj, "three slices", threads=2)
    assert base["cores"] == 2 and base["single_thread"]["cores"] == 1
    assert check["problems"] == 3 and check["thresholds_identical"] == 3
    assert check["max_rel_objective_error"] == 0.0


def test_summarize_sq_per_dispatch_and_per_wavefront(tmp_path):
    """SQ counters: summed over a counter's instances within a dispatch,
    averaged over dispatches; runtime kernels and the issue-rate probe left
    out; instructions per wavefront from SQ_WAVES."""
    rows = ["Correlation_Id,Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    for disp, scale in ((1, 1.0), (2, 3.0)):
        for inst in range(2):  # two instances of each counter per dispatch
            rows.append(f"{disp},{disp},\"ts::k_morph<false, 0>(int)\",SQ_INSTS_VALU,{500 * scale}")
            rows.append(f"{disp},{disp},\"ts::k_morph<false, 0>(int)\",SQ_WAVES,{5 * scale}")
    rows.append("3,3,void ts::k_issue<1>(float),SQ_INSTS_VALU,7")
    rows.append("4,4,__amd_rocclr_copyBuffer,SQ_INSTS_VALU,9")
    d = tmp_path / "sq"
    d.mkdir()
    (d / "pmc_counter_collection.csv").write_text("\n".join(rows) + "\n")
    out = bench.summarize_sq([str(d)], "hdr")
    assert out.startswith("hdr\n")
    assert "k_issue" not in out and "copyBuffer" not in out
    assert "SQ_INSTS_VALU=2000" in out and "SQ_WAVES=20" in out  # (1000 + 3000) / 2, (10 + 30) / 2
    assert "per wavefront: VALU=100.0" in out
