"""The C-ABI library on the CPU: it loads, exports every symbol include/ts.h
declares, sizes workspaces, and rejects bad arguments before any launch
(no GPU is touched by these calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ts.h")
LIB = os.path.join(ROOT, "paper_2012_10684_amd", "libts.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(ts_[a-z_0-9]+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libts.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_path():
    names = declared_functions()
    for n in ("ts_histogram", "ts_prefix", "ts_threshold_search", "ts_label", "ts_label_sets",
              "ts_search_workspace_bytes", "ts_segment", "ts_segment_workspace_bytes", "ts_threshold_search_noalloc",
              "ts_last_error", "ts_abi_version"):
        assert n in names, names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for n in declared_functions():
        assert n in exported, f"{n} declared in ts.h but not exported"
        getattr(lib, n)


class Binning(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32), ("hi", ctypes.c_int32), ("nbins", ctypes.c_int32)]


class Batch(ctypes.Structure):
    _fields_ = [("vox", ctypes.c_void_p), ("offs", ctypes.c_void_p), ("nseg", ctypes.c_int32),
                ("total", ctypes.c_int64)]


def _bind(lib):
    P, i32, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    lib.ts_histogram.argtypes = [Batch, Binning, P, P, P]
    lib.ts_prefix.argtypes = [P, i32, i32, i32, P, P, P, P]
    lib.ts_search_workspace_bytes.argtypes = [i32, i32, i32, i32, i32]
    lib.ts_search_workspace_bytes.restype = sz
    lib.ts_threshold_search.argtypes = [P, P, i32, i32, i32, i32, P, i32, P, sz, P, P, P, P, P]
    lib.ts_label.argtypes = [Batch, Binning, P, i32, P, P, P]
    lib.ts_label_sets.argtypes = [Batch, Binning, i32, P, i32, P, P, P]
    lib.ts_log2_f32.argtypes = [P, P, ctypes.c_int64, P]
    lib.ts_issue_rate.argtypes = [i32, i32, i32, P, P]
    lib.ts_histogram2d.argtypes = [Batch, i32, i32, Binning, P, P]
    lib.ts_search2d_workspace_bytes.argtypes = [i32, i32, i32]
    lib.ts_search2d_workspace_bytes.restype = sz
    lib.ts_threshold_search2d.argtypes = [P, i32, i32, i32, P, P, sz, P, P, P, P]
    lib.ts_open2d_workspace_bytes.argtypes = [i32, i32, i32]
    lib.ts_open2d_workspace_bytes.restype = sz
    lib.ts_open2d.argtypes = [Batch, i32, i32, Binning, i32, P, sz, P, P, P, P]
    lib.ts_search_dp_workspace_bytes.argtypes = [i32, i32, i32, i32]
    lib.ts_search_dp_workspace_bytes.restype = sz
    lib.ts_threshold_search_dp.argtypes = [P, P, i32, i32, i32, i32, P, P, sz, P, P, P, P]
    lib.ts_threshold_search_noalloc.argtypes = [P, P, i32, i32, i32, i32, P, i32, P, P, P, P, P]
    lib.ts_segment_workspace_bytes.argtypes = [i32, i32, i32, i32, i32, i32]
    lib.ts_segment_workspace_bytes.restype = sz
    lib.ts_segment.argtypes = [Batch, Binning, i32, i32, P, i32, P, P, P, P, P, P, sz, P, P]
    lib.ts_last_error.restype = ctypes.c_char_p
    return lib


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first


def qs(*v):
    """[host] array of q values."""
    return ctypes.cast((ctypes.c_double * len(v))(*v), ctypes.c_void_p)


def test_abi_version(lib):
    lib.ts_abi_version.restype = ctypes.c_int32
    assert lib.ts_abi_version() == 3


def test_workspace_sizes(lib):
    _bind(lib)
    ws = lib.ts_search_workspace_bytes
    assert ws(1, 4096, 1, 1, 0) > 0
    assert ws(300, 256, 2, 1, 0) >= 300 * 256 * 8  # head + tail rows
    assert 0 < ws(1, 1024, 3, 1, 0) < ws(1, 1024, 3, 1, 2)  # FP32 k = 3 builds its rows in LDS
    assert ws(1, 1024, 3, 1, 2) >= 2 * 1024 * 1024 * 8  # FP64 rows
    assert ws(10, 256, 2, 1, 0) > ws(5, 256, 2, 1, 0)
    assert ws(100, 256, 2, 3, 0) == ws(300, 256, 2, 1, 0)  # nq x nseg problems
    # the plain forms (FP64: mode 3, FP32: mode 5) keep one best per block of tuples
    assert ws(1, 1024, 3, 1, 5) == ws(1, 1024, 3, 1, 3) > 0
    for bad in [(-1, 256, 1, 1, 0), (1, 1, 1, 1, 0), (1, 4097, 1, 1, 0), (1, 256, 0, 1, 0), (1, 256, 4, 1, 0),
                (1, 256, 1, 1, 6), (1, 256, 1, 1, 7), (1, 256, 1, 0, 0), (1, 256, 1, 9, 0)]:
        assert ws(*bad) == 0, bad
    dpws = lib.ts_search_dp_workspace_bytes
    assert dpws(1, 1024, 4, 1) == 4 * 1024 * 8 and dpws(300, 256, 2, 3) == 2 * 900 * 256 * 8
    for bad in [(-1, 256, 2, 1), (1, 1, 1, 1), (1, 4097, 1, 1), (1, 256, 0, 1), (1, 256, 17, 1), (1, 256, 2, 0)]:
        assert dpws(*bad) == 0, bad


@pytest.mark.parametrize("case,expect", [
    ("hist_neg_nseg", 1), ("hist_bad_bins", 1), ("hist_lo_gt_hi", 1), ("hist_null", 1), ("hist_bad_tune", 1),
    ("prefix_q0", 1), ("prefix_qnan", 1), ("prefix_bins", 1), ("prefix_null", 1), ("prefix_nq0", 1),
    ("prefix_nq9", 1), ("prefix_qarr_null", 1), ("prefix_second_q_bad", 1),
    ("search_k0", 1), ("search_k4", 1), ("search_qneg", 1), ("search_mode", 1), ("search_ws", 3),
    ("search_bins_lt_k1", 1), ("search_null", 1), ("search_nq0", 1), ("search_nq9", 1), ("search_qnan_in_batch", 1),
    ("label_k", 1), ("label_null", 1), ("label_total_without_seg", 1),
    ("sets_zero", 1), ("sets_five", 1), ("sets_null_array", 1), ("sets_null_entry", 1), ("sets_k", 1),
    ("log2_neg", 1), ("log2_null", 1), ("issue_op", 1), ("issue_blocks", 1), ("issue_null", 1),
    ("h2d_bins", 1), ("h2d_width", 1), ("h2d_total", 1), ("h2d_null", 1),
    ("s2d_bins", 1), ("s2d_q", 1), ("s2d_ws", 3), ("s2d_null", 1),
    ("open_bins", 1), ("open_radius", 1), ("open_radius_neg", 1), ("open_total", 1), ("open_no_output", 1),
    ("open_ws", 3), ("open_height", 1), ("open_huge", 1),
    ("dp_k0", 1), ("dp_k17", 1), ("dp_bins_lt_k1", 1), ("dp_q", 1), ("dp_ws", 3), ("dp_null", 1), ("dp_misaligned", 1),
    ("seg_k4", 1), ("seg_ws", 3), ("seg_nq5_labels", 1), ("seg_null_hist", 1), ("seg_null_out_entry", 1),
    ("seg_bad_parts", 1), ("seg_bad_block", 1), ("seg_q", 1), ("seg_bins", 3),
    ("noalloc_k0", 1), ("noalloc_null", 1), ("noalloc_beyond_scratch", 3),
])
def test_argument_errors(lib, case, expect):
    _bind(lib)
    ok_bin = Binning(-1024, 3071, 1024)
    b1 = Batch(FAKE, FAKE, 1, 10)
    sx = None
    T = ctypes.c_void_p
    if case == "hist_neg_nseg":
        st = lib.ts_histogram(Batch(FAKE, FAKE, -1, 0), ok_bin, FAKE, None, sx)
    elif case == "hist_bad_bins":
        st = lib.ts_histogram(b1, Binning(0, 10, 4097), FAKE, None, sx)
    elif case == "hist_lo_gt_hi":
        st = lib.ts_histogram(b1, Binning(10, 0, 16), FAKE, None, sx)
    elif case == "hist_null":
        st = lib.ts_histogram(Batch(None, FAKE, 1, 10), ok_bin, FAKE, None, sx)
    elif case == "hist_bad_tune":
        tune = (ctypes.c_int32 * 12)(100, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0)  # block not a multiple of 64
        st = lib.ts_histogram(b1, ok_bin, FAKE, ctypes.cast(tune, T), sx)
    elif case == "prefix_q0":
        st = lib.ts_prefix(FAKE, 1, 256, 1, qs(0.0), FAKE, FAKE, sx)
    elif case == "prefix_qnan":
        st = lib.ts_prefix(FAKE, 1, 256, 1, qs(float("nan")), FAKE, FAKE, sx)
    elif case == "prefix_bins":
        st = lib.ts_prefix(FAKE, 1, 1, 1, qs(0.8), FAKE, FAKE, sx)
    elif case == "prefix_null":
        st = lib.ts_prefix(None, 1, 256, 1, qs(0.8), FAKE, FAKE, sx)
    elif case == "prefix_nq0":
        st = lib.ts_prefix(FAKE, 1, 256, 0, qs(0.8), FAKE, FAKE, sx)
    elif case == "prefix_nq9":
        st = lib.ts_prefix(FAKE, 1, 256, 9, qs(*([0.8] * 9)), FAKE, FAKE, sx)
    elif case == "prefix_qarr_null":
        st = lib.ts_prefix(FAKE, 1, 256, 1, None, FAKE, FAKE, sx)
    elif case == "prefix_second_q_bad":
        st = lib.ts_prefix(FAKE, 1, 256, 2, qs(0.8, -1.0), FAKE, FAKE, sx)
    elif case.startswith("search_"):
        k = {"search_k0": 0, "search_k4": 4}.get(case, 2)
        q = {"search_qneg": (-0.5,), "search_qnan_in_batch": (0.5, 1.0, float("nan"))}.get(case, (0.8,))
        nq = {"search_nq0": 0, "search_nq9": 9}.get(case, len(q))
        if case == "search_nq9":
            q = (0.8,) * 9
        mode = 9 if case == "search_mode" else 0
        L = 2 if case == "search_bins_lt_k1" else 256
        ws_bytes = 16 if case == "search_ws" else 1 << 40
        P = None if case == "search_null" else FAKE
        st = lib.ts_threshold_search(P, FAKE, 1, L, k, nq, qs(*q), mode, FAKE, ws_bytes, FAKE, FAKE, FAKE, None, sx)
    elif case == "label_k":
        st = lib.ts_label(b1, ok_bin, FAKE, 0, FAKE, None, sx)
    elif case == "label_null":
        st = lib.ts_label(b1, ok_bin, None, 1, FAKE, None, sx)
    elif case == "label_total_without_seg":
        st = lib.ts_label(Batch(None, None, 0, 5), ok_bin, FAKE, 1, FAKE, None, sx)
    elif case.startswith("h2d_"):
        b = Batch(FAKE, FAKE, 2, 2 * 4 * 5)
        binning = Binning(-1024, 3071, 512 if case == "h2d_bins" else 256)
        W = 5000 if case == "h2d_width" else 5
        if case == "h2d_total":
            b = Batch(FAKE, FAKE, 2, 39)
        st = lib.ts_histogram2d(b, 4, W, binning, None if case == "h2d_null" else FAKE, sx)
    elif case.startswith("s2d_"):
        L = 257 if case == "s2d_bins" else 64
        q = qs(-1.0) if case == "s2d_q" else qs(0.8)
        ws_bytes = 8 if case == "s2d_ws" else 1 << 40
        st = lib.ts_threshold_search2d(None if case == "s2d_null" else FAKE, 3, L, 1, q, FAKE, ws_bytes, FAKE,
                                       FAKE, FAKE, sx)
    elif case.startswith("open_"):
        b = Batch(FAKE, FAKE, 2, 2 * 6 * 7)
        binning = Binning(-1024, 3071, 512 if case == "open_bins" else 256)
        r = {"open_radius": 33, "open_radius_neg": -1}.get(case, 10)
        if case == "open_total":
            b = Batch(FAKE, FAKE, 2, 83)
        Hh = 0 if case == "open_height" else 6
        Ww = 7
        if case == "open_huge":  # one image of 2^30 pixels: beyond TS_MORPH_MAX_PIXELS
            Hh, Ww = 1 << 15, 1 << 15
            b = Batch(FAKE, FAKE, 1, Hh * Ww)
        ws_bytes = 10 if case == "open_ws" else 1 << 31
        outs = (None, None) if case == "open_no_output" else (FAKE, None)
        st = lib.ts_open2d(b, Hh, Ww, binning, r, FAKE, ws_bytes, outs[0], outs[1], None, sx)
    elif case.startswith("dp_"):
        k = {"dp_k0": 0, "dp_k17": 17}.get(case, 5)
        L = 5 if case == "dp_bins_lt_k1" else 512
        q = qs(0.0) if case == "dp_q" else qs(0.8)
        ws_bytes = 8 if case == "dp_ws" else 1 << 40
        ws = ctypes.c_void_p(0x1004) if case == "dp_misaligned" else FAKE
        st = lib.ts_threshold_search_dp(None if case == "dp_null" else FAKE, FAKE, 2, L, k, 1, q, ws, ws_bytes, FAKE,
                                        FAKE, FAKE, sx)
    elif case.startswith("seg_"):
        k = 4 if case == "seg_k4" else 2
        nq = 5 if case == "seg_nq5_labels" else 2
        q = qs(*([0.8] * nq)) if case != "seg_q" else qs(0.8, 0.0)
        binning = Binning(-1024, 3071, 2000 if case == "seg_bins" else 256)
        tune = None
        if case in ("seg_bad_parts", "seg_bad_block"):
            vals = [0] * 12
            vals[10 if case == "seg_bad_parts" else 11] = 65 if case == "seg_bad_parts" else 384
            tune = ctypes.cast((ctypes.c_int32 * 12)(*vals), T)
        outp = (T * 5)(*([FAKE.value] * 5))
        if case == "seg_null_out_entry":
            outp[1] = None
        # 2000 bins with k = 2 run the separate passes: valid sizes, the workspace too small
        ws_bytes = 16 if case in ("seg_ws", "seg_bins") else 1 << 40
        st = lib.ts_segment(b1, binning, k, nq, q, 0, None if case == "seg_null_hist" else FAKE, FAKE, FAKE, FAKE,
                            ctypes.cast(outp, T), FAKE, ws_bytes, tune, sx)
    elif case.startswith("noalloc_"):
        k = 0 if case == "noalloc_k0" else 2
        P = None if case == "noalloc_null" else FAKE
        n = 20000 if case == "noalloc_beyond_scratch" else 2
        tune = (ctypes.c_int32 * 12)(0, 0, 0, 0, 0, 0, 0, 0, 2, 0, 0, 0)  # one launch per phase: uses scratch
        st = lib.ts_threshold_search_noalloc(P, FAKE, n, 256, k, 1, qs(0.8), 0, FAKE, FAKE, FAKE,
                                             ctypes.cast(tune, T), sx)
    elif case == "log2_neg":
        st = lib.ts_log2_f32(FAKE, FAKE, -1, sx)
    elif case == "log2_null":
        st = lib.ts_log2_f32(None, FAKE, 10, sx)
    elif case == "issue_op":
        st = lib.ts_issue_rate(3, 8, 8, FAKE, sx)
    elif case == "issue_blocks":
        st = lib.ts_issue_rate(0, 0, 8, FAKE, sx)
    elif case == "issue_null":
        st = lib.ts_issue_rate(1, 8, 8, None, sx)
    elif case.startswith("sets_"):
        n = {"sets_zero": 0, "sets_five": 5}.get(case, 2)
        thr = (T * 5)(*([FAKE.value] * 5))
        outp = (T * 5)(*([FAKE.value] * 5))
        if case == "sets_null_entry":
            outp[1] = None
        arr = None if case == "sets_null_array" else ctypes.cast(thr, T)
        st = lib.ts_label_sets(b1, ok_bin, n, arr, 17 if case == "sets_k" else 2, ctypes.cast(outp, T), None, sx)
    assert st == expect, (case, st, lib.ts_last_error())
    assert lib.ts_last_error(), "an error text must be set"


def test_empty_batch_is_a_no_op(lib):
    _bind(lib)
    ok_bin = Binning(-1024, 3071, 256)
    assert lib.ts_histogram(Batch(None, None, 0, 0), ok_bin, None, None, None) == 0
    assert lib.ts_label(Batch(None, None, 0, 0), ok_bin, None, 1, None, None, None) == 0
    assert lib.ts_label_sets(Batch(None, None, 0, 0), ok_bin, 3, None, 2, None, None, None) == 0
    assert lib.ts_log2_f32(None, None, 0, None) == 0
    assert lib.ts_histogram2d(Batch(None, None, 0, 0), 4, 4, ok_bin, None, None) == 0
    assert lib.ts_threshold_search2d(None, 0, 64, 1, qs(0.8), None, 0, None, None, None, None) == 0
    assert lib.ts_threshold_search_dp(None, None, 0, 1024, 4, 1, qs(0.8), None, 0, None, None, None, None) == 0
    assert lib.ts_open2d(Batch(None, None, 0, 0), 8, 8, ok_bin, 10, None, 0, None, None, None, None) == 0
    assert lib.ts_open2d_workspace_bytes(3, 512, 512) == 3 * 512 * 512
    assert lib.ts_prefix(None, 0, 256, 1, qs(0.8), None, None, None) == 0
    assert lib.ts_threshold_search(None, None, 0, 256, 2, 2, qs(0.8, 1.5), 0, None, 0, None, None, None, None,
                                   None) == 0
    assert lib.ts_threshold_search_noalloc(None, None, 0, 256, 2, 2, qs(0.8, 1.5), 0, None, None, None, None,
                                           None) == 0
    assert lib.ts_segment(Batch(None, None, 0, 0), ok_bin, 2, 1, qs(0.8), 0, None, None, None, None, None, None, 0,
                          None, None) == 0


def test_segment_workspace_sizes(lib):
    _bind(lib)
    ws = lib.ts_segment_workspace_bytes
    # fused (k <= 2): tickets + partial histograms of at most 1024 workgroups; below 1024 problems at least
    # what the separate passes need
    assert ws(1, 4096, 1, 1, 0, 1) >= 256 + 4096 * 4 * 64
    assert ws(1, 4096, 1, 1, 0, 1) >= 2 * 4096 * 8 + lib.ts_search_workspace_bytes(1, 4096, 1, 1, 0)
    assert ws(22844, 256, 2, 1, 0, 1) == ((22844 * 8 + 255) // 256) * 256 + 256 * 4 * 1024
    # separate passes (k = 3, or FP64): P, Q and the search workspace
    assert ws(1, 1024, 3, 1, 0, 1) >= 2 * 1024 * 8 + lib.ts_search_workspace_bytes(1, 1024, 3, 1, 0)
    assert ws(2, 256, 2, 1, 2, 1) >= 2 * 2 * 256 * 8
    for bad in [(-1, 256, 2, 1, 0, 1), (1, 1, 1, 1, 0, 1), (1, 256, 4, 1, 0, 1), (1, 256, 2, 5, 0, 1),
                (1, 256, 2, 9, 0, 0), (1, 256, 2, 1, 9, 1)]:
        assert ws(*bad) == 0, bad
