"""CPU FP64 oracle for maximum-Tsallis-entropy thresholding (arXiv 2012.10684).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library never calls it and shares no code with it; the two meet only in the
seeded input generator, which holds none of the method's arithmetic.

All arithmetic lives in ``oracle.c`` (plain C, FP64, built with gcc without
fast-math); this module only marshals numpy arrays through ctypes.

Functions and the passages they follow:
  bin_map / histogram -- Pre-processing section (linear map of levels onto L
                         gray levels) and Thresholding section (histogram as
                         the measurement space).
  prefix              -- Tsallis-entropy section: p_i = c_i/N, P(t) = sum p_i,
                         Q(t) = sum p_i^q (left-to-right sums).
  search / objective  -- Tsallis-entropy section: class entropies H_j, the
                         pseudo-additive objective and its arg max, extended to
                         k thresholds by applying the composition rule
                         recursively.
  label               -- Algorithm 1 (thresholding kernel function),
                         generalised to k thresholds.
  mean3x3 / histogram2d / search2d / objective2d (``oracle2d.c``)
                      -- Tsallis-entropy section, two-dimensional form: the
                         3x3 average image, the 2D histogram of (gray level,
                         average gray level), the class entropies over
                         quadrants 1 and 3 and the arg max over (t, s).
  morph / opening (``morph.c``)
                      -- Morphology section: gray-scale erosion and dilation
                         by a flat disk, the opening and the residue
                         original - opened.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRC2 = os.path.join(_HERE, "oracle2d.c")
_SRC3 = os.path.join(_HERE, "morph.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODE_DIRECT = 0
MODE_PREFIX = 1
MODE_KAPUR = 2
COMP_RECURSIVE = 0  # T <- T + S_j + (1-q) T S_j
COMP_SUMPROD = 1    # sum_j S_j + (1-q) prod_j S_j

OK = 0
DEGENERATE = 1
EMPTY = 2
BADARG = 3


def compile_source(src, out: str) -> str:
    """Compile C source(s) into a shared library with gcc (-O2, IEEE
    semantics, no contraction).  Used for the oracle itself and, by the
    tests, for deliberately mutated copies of oracle.c."""
    tmp = out + ".tmp"
    srcs = [src] if isinstance(src, str) else list(src)
    subprocess.run(
        ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
         "-ffp-contract=off", "-Wall", "-Wextra", "-o", tmp] + srcs + ["-lm"],
        check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so."""
    if force or _stale():
        compile_source([_SRC, _SRC2, _SRC3], _LIB)
    return _LIB


def _stale() -> bool:
    return not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
        os.path.getmtime(p) for p in (_SRC, _SRC2, _SRC3))


def load_library(path: str):
    """Load an oracle-compatible shared library (the tests load mutants)."""
    return _bind(ctypes.CDLL(path))


def _bind(lib):
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.or_bin.argtypes = [i32, i32, i32, i32]
    lib.or_bin.restype = i32
    lib.or_bin_map.argtypes = [P, i64, i32, i32, i32, P]
    lib.or_bin_map.restype = None
    lib.or_histogram.argtypes = [P, i64, i32, i32, i32, P]
    lib.or_histogram.restype = None
    lib.or_prefix.argtypes = [P, i32, f64, P, P]
    lib.or_prefix.restype = None
    lib.or_search.argtypes = [P, i32, i32, f64, i32, P, P, P]
    lib.or_search.restype = i32
    lib.or_objective.argtypes = [P, i32, i32, f64, i32, P]
    lib.or_objective.restype = f64
    lib.or_search_c.argtypes = [P, i32, i32, f64, i32, i32, P, P, P]
    lib.or_search_c.restype = i32
    lib.or_objective_c.argtypes = [P, i32, i32, f64, i32, i32, P]
    lib.or_objective_c.restype = f64
    lib.or_label.argtypes = [P, i64, i32, i32, i32, P, i32, P]
    lib.or_label.restype = None
    if hasattr(lib, "or_search_dp"):
        lib.or_search_dp.argtypes = [P, i32, i32, f64, i32, P, P]
        lib.or_search_dp.restype = i32
    if hasattr(lib, "or2_search"):  # mutated copies of oracle.c alone lack the 2-D part
        lib.or2_mean3x3.argtypes = [P, i32, i32, P]
        lib.or2_mean3x3.restype = None
        lib.or2_histogram.argtypes = [P, i32, i32, i32, i32, i32, P]
        lib.or2_histogram.restype = None
        lib.or2_objective.argtypes = [P, i32, f64, i32, i32, i32]
        lib.or2_objective.restype = f64
        lib.or2_search.argtypes = [P, i32, f64, i32, P, P, P, P]
        lib.or2_search.restype = i32
    if hasattr(lib, "or_open"):  # mutated copies of the other sources alone lack it
        lib.or_morph.argtypes = [P, i32, i32, i32, i32, P]
        lib.or_morph.restype = None
        lib.or_open.argtypes = [P, i32, i32, i32, P, P, P]
        lib.or_open.restype = None
    return lib


_lib = None


def _load():
    global _lib
    if _lib is None:
        if _stale():
            build(force=True)
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def bin_of(v: int, lo: int, hi: int, L: int, lib=None) -> int:
    return int((lib or _load()).or_bin(int(v), int(lo), int(hi), int(L)))


def bin_map(vox: np.ndarray, lo: int, hi: int, L: int, lib=None) -> np.ndarray:
    v = np.ascontiguousarray(vox, dtype=np.int16).reshape(-1)
    out = np.empty(v.size, dtype=np.int32)
    (lib or _load()).or_bin_map(_ptr(v), v.size, lo, hi, L, _ptr(out))
    return out


def histogram(vox: np.ndarray, lo: int, hi: int, L: int, lib=None) -> np.ndarray:
    v = np.ascontiguousarray(vox, dtype=np.int16).reshape(-1)
    h = np.empty(L, dtype=np.uint32)
    (lib or _load()).or_histogram(_ptr(v), v.size, lo, hi, L, _ptr(h))
    return h


def prefix(hist: np.ndarray, q: float, lib=None):
    h = np.ascontiguousarray(hist, dtype=np.uint32)
    L = h.size
    P = np.empty(L, dtype=np.float64)
    Q = np.empty(L, dtype=np.float64)
    (lib or _load()).or_prefix(_ptr(h), L, float(q), _ptr(P), _ptr(Q))
    return P, Q


class SearchResult:
    """Oracle outcome for one problem: thresholds, objective S*, runner-up S."""

    __slots__ = ("thr", "obj", "second", "status")

    def __init__(self, thr, obj, second, status):
        self.thr = thr
        self.obj = obj
        self.second = second
        self.status = status

    def rel_gap(self) -> float:
        """(S* - S_2) / |S*|: relative gap to the best tuple other than thr."""
        if self.status != OK or not np.isfinite(self.second):
            return float("inf")
        if self.obj == 0.0:
            return 0.0 if self.second == 0.0 else float("inf")
        return (self.obj - self.second) / abs(self.obj)

    def __repr__(self):
        return f"SearchResult(thr={self.thr.tolist()}, obj={self.obj!r}, second={self.second!r}, status={self.status})"


def search(hist: np.ndarray, k: int, q: float, mode: int = MODE_PREFIX, lib=None,
           comp: int = COMP_RECURSIVE) -> SearchResult:
    """Exhaustive first arg max; comp selects the composition of the class
    entropies (COMP_RECURSIVE: the pseudo-additive rule applied recursively;
    COMP_SUMPROD: sum of S_j + (1-q) product of S_j)."""
    h = np.ascontiguousarray(hist, dtype=np.uint32)
    thr = np.empty(k, dtype=np.int32)
    best = ctypes.c_double()
    second = ctypes.c_double()
    st = (lib or _load()).or_search_c(_ptr(h), h.size, int(k), float(q), int(mode), int(comp), _ptr(thr),
                                      ctypes.byref(best), ctypes.byref(second))
    if st == BADARG:
        raise ValueError(f"oracle.search: bad arguments L={h.size} k={k} q={q} mode={mode}")
    return SearchResult(thr, best.value, second.value, st)


def search_dp(hist: np.ndarray, k: int, q: float, mode: int = MODE_PREFIX, lib=None) -> SearchResult:
    """Arg max by dynamic programming over class boundaries (prefix or Kapur
    mode): the same objective and tie rule as search(), for numbers of
    thresholds the exhaustive search cannot reach; second is not computed."""
    h = np.ascontiguousarray(hist, dtype=np.uint32)
    thr = np.empty(k, dtype=np.int32)
    best = ctypes.c_double()
    st = (lib or _load()).or_search_dp(_ptr(h), h.size, int(k), float(q), int(mode), _ptr(thr), ctypes.byref(best))
    if st == BADARG:
        raise ValueError(f"oracle.search_dp: bad arguments L={h.size} k={k} q={q} mode={mode}")
    return SearchResult(thr, best.value, float("nan"), st)


def objective(hist: np.ndarray, thr, q: float, mode: int = MODE_PREFIX, lib=None,
              comp: int = COMP_RECURSIVE) -> float:
    h = np.ascontiguousarray(hist, dtype=np.uint32)
    t = np.ascontiguousarray(np.asarray(thr, dtype=np.int32).reshape(-1))
    return float((lib or _load()).or_objective_c(_ptr(h), h.size, t.size, float(q), int(mode), int(comp), _ptr(t)))


def label(vox: np.ndarray, lo: int, hi: int, L: int, thr, lib=None) -> np.ndarray:
    v = np.ascontiguousarray(vox, dtype=np.int16)
    t = np.ascontiguousarray(np.asarray(thr, dtype=np.int32).reshape(-1))
    out = np.empty(v.shape, dtype=np.uint8)
    (lib or _load()).or_label(_ptr(v), v.size, lo, hi, L, _ptr(t), t.size, _ptr(out))
    return out


def segment(vox: np.ndarray, lo: int, hi: int, L: int, k: int, q: float, mode: int = MODE_PREFIX, lib=None):
    """The whole path for one problem: histogram -> arg max -> labels."""
    h = histogram(vox, lo, hi, L, lib=lib)
    r = search(h, k, q, mode, lib=lib)
    lab = label(vox, lo, hi, L, r.thr, lib=lib)
    return h, r, lab


# ------------------------------------------------------------------ 2-D form

def mean3x3(f: np.ndarray, lib=None) -> np.ndarray:
    """Floor of the 3x3 mean of an integer image (edge pixels repeated)."""
    f = np.ascontiguousarray(f, dtype=np.int32)
    H, W = f.shape
    g = np.empty_like(f)
    (lib or _load()).or2_mean3x3(_ptr(f), H, W, _ptr(g))
    return g


def histogram2d(img: np.ndarray, lo: int, hi: int, L: int, lib=None) -> np.ndarray:
    """2D histogram [L, L] (row = gray level, column = 3x3 average gray level)
    of one int16 image."""
    img = np.ascontiguousarray(img, dtype=np.int16)
    H, W = img.shape
    h = np.empty((L, L), dtype=np.uint32)
    (lib or _load()).or2_histogram(_ptr(img), H, W, int(lo), int(hi), int(L), _ptr(h))
    return h


def objective2d(h2: np.ndarray, t: int, s: int, q: float, mode: int = MODE_PREFIX, lib=None) -> float:
    h2 = np.ascontiguousarray(h2, dtype=np.uint32)
    return float((lib or _load()).or2_objective(_ptr(h2), h2.shape[0], float(q), int(mode), int(t), int(s)))


def search2d(h2: np.ndarray, q: float, mode: int = MODE_PREFIX, lib=None) -> SearchResult:
    """Arg max of the two-dimensional objective over (t, s); thr = [t, s]."""
    h2 = np.ascontiguousarray(h2, dtype=np.uint32)
    L = h2.shape[0]
    t, s_ = ctypes.c_int32(), ctypes.c_int32()
    obj, sec = ctypes.c_double(), ctypes.c_double()
    st = (lib or _load()).or2_search(_ptr(h2), L, float(q), int(mode), ctypes.byref(t), ctypes.byref(s_),
                                      ctypes.byref(obj), ctypes.byref(sec))
    return SearchResult(np.array([t.value, s_.value], dtype=np.int32), obj.value, sec.value, int(st))


def morph(f: np.ndarray, r: int, take_max: bool, lib=None) -> np.ndarray:
    """Gray-scale erosion (take_max False) or dilation by the disk of radius r
    (pixels outside the image take no part)."""
    f = np.ascontiguousarray(f, dtype=np.int32)
    H, W = f.shape
    out = np.empty_like(f)
    (lib or _load()).or_morph(_ptr(f), H, W, int(r), int(bool(take_max)), _ptr(out))
    return out


def opening(f: np.ndarray, r: int, lib=None):
    """(opened, residue = f - opened) of the gray image f by the disk of radius r."""
    f = np.ascontiguousarray(f, dtype=np.int32)
    H, W = f.shape
    tmp, opened, residue = np.empty_like(f), np.empty_like(f), np.empty_like(f)
    (lib or _load()).or_open(_ptr(f), H, W, int(r), _ptr(tmp), _ptr(opened), _ptr(residue))
    return opened, residue


def gray(img: np.ndarray, lo: int, hi: int, L: int, lib=None) -> np.ndarray:
    """Gray levels of an int16 image under the bin map (same shape)."""
    v = np.ascontiguousarray(img, dtype=np.int16)
    return bin_map(v.reshape(-1), lo, hi, L, lib=lib).reshape(v.shape)
