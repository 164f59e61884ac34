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
    for f in ("k_label.hip", "common.h"):
        shutil.copy(os.path.join(src, f), dst / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    rec = {"k_label.hip": {"src_sha": bench.src_hash("k_label.hip"), "workload": "volume300",
                           "bytes_per_launch": 123.0}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    return dst


def test_traffic_used_for_its_source_and_workload(tree):
    assert bench.load_traffic("k_label.hip", "volume300") == 123.0
    assert bench.load_traffic("k_label.hip", "volume600") is None  # another workload
    assert bench.load_traffic("k_histogram.hip", "volume300") is None  # no record


@pytest.mark.parametrize("changed", ["k_label.hip", "common.h"])
def test_traffic_dropped_once_the_kernel_changes(tree, changed):
    with open(tree / changed, "a") as f:
        f.write("\n// edited\n")
    assert bench.load_traffic("k_label.hip", "volume300") is None


def test_cpu_baseline_repeats_a_short_sample(monkeypatch):
    monkeypatch.setattr(bench, "CPU_MIN_S", 0.3)
    vol = synth.workload_slice(0)[None]
    base, check = bench.cpu_baseline(vol, 1, bench.WORKLOADS["slice"], np.array([[[0]]]), np.array([[1.0]]))
    passes = int(base["sample"].split(" pass")[0].rsplit(" ", 1)[-1])
    assert passes >= 2, base
    assert np.isfinite(base["value"]) and base["value"] > 0 and base["cores"] == 1
    assert check["problems"] == 1  # the agreement check covers the first pass only
