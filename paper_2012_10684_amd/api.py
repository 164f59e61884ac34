"""Python binding of libts (include/ts.h): argument marshalling only.

Every step of the path runs in the HIP library; PyTorch provides device
memory (tensors) and the stream.  There is no fallback: if ``libts.so`` has
not been built, importing this module raises ImportError.

Functions mirror the C ABI:
  histogram(batch, binning)          -> uint32 counts [nseg, L] (int32 storage)
  prefix(hist, q)                    -> P, Q float64 [nseg, L]
  threshold_search(P, Q, k, q, mode) -> thr int32 [nseg, k], obj float64 [nseg], status int32 [nseg]
  (q may also be a sequence of up to MAX_Q values: Q, thr, obj and status
  then get a leading [nq] dimension and every q is handled by one launch)
  label(batch, binning, thr, k)      -> one uint8 tensor per problem
  label_sets(batch, binning, thrs, k) -> one list of uint8 tensors per threshold set
plus ``Batch`` (the device segment table) and ``segment`` (the four calls in
order).
"""
from __future__ import annotations

import contextlib
import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TS_LIBRARY", os.path.join(_HERE, "libts.so"))

ABI_VERSION = 3
MAX_Q = 8
TS_OK, TS_ERR_INVALID_ARG, TS_ERR_UNSUPPORTED, TS_ERR_WORKSPACE, TS_ERR_HIP = 0, 1, 2, 3, 4
SEARCH_FP32_TIECHECK, SEARCH_FP32_ONLY, SEARCH_FP64, SEARCH_PLAIN, SEARCH_SUMPROD, SEARCH_PLAIN_FP32 = 0, 1, 2, 3, 4, 5
PROBLEM_OK, PROBLEM_DEGENERATE, PROBLEM_EMPTY, PROBLEM_SYNC_FAILED = 0, 1, 2, 3


class Binning(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32), ("hi", ctypes.c_int32), ("nbins", ctypes.c_int32)]

    def __repr__(self):
        return f"Binning(lo={self.lo}, hi={self.hi}, nbins={self.nbins})"


class _Batch(ctypes.Structure):
    _fields_ = [("vox", ctypes.c_void_p), ("offs", ctypes.c_void_p), ("nseg", ctypes.c_int32),
                ("total", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "hist_block", "hist_replicas", "hist_wg_per_cu", "label_block", "label_vecs",
        "search_cols", "search_rows", "min_chunk", "search_path", "search_block", "segment_parts",
        "segment_block")]

    @classmethod
    def from_dict(cls, d: Optional[dict]):
        t = cls()
        for k, v in (d or {}).items():
            setattr(t, k, int(v))
        return t

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class TsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libts status {status}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    lib.ts_histogram.argtypes = [_Batch, Binning, P, P, P]
    lib.ts_prefix.argtypes = [P, i32, i32, i32, P, P, P, P]
    lib.ts_search_workspace_bytes.argtypes = [i32, i32, i32, i32, i32]
    lib.ts_search_workspace_bytes.restype = sz
    lib.ts_threshold_search.argtypes = [P, P, i32, i32, i32, i32, P, i32, P, sz, P, P, P, P, P]
    lib.ts_threshold_search_noalloc.argtypes = [P, P, i32, i32, i32, i32, P, i32, P, P, P, P, P]
    lib.ts_segment_workspace_bytes.argtypes = [i32, i32, i32, i32, i32, i32]
    lib.ts_segment_workspace_bytes.restype = sz
    lib.ts_segment.argtypes = [_Batch, Binning, i32, i32, P, i32, P, P, P, P, P, P, sz, P, P]
    lib.ts_label.argtypes = [_Batch, Binning, P, i32, P, P, P]
    lib.ts_label_sets.argtypes = [_Batch, Binning, i32, P, i32, P, P, P]
    lib.ts_log2_f32.argtypes = [P, P, i64, P]
    lib.ts_issue_rate.argtypes = [i32, i32, i32, P, P]
    lib.ts_histogram2d.argtypes = [_Batch, i32, i32, Binning, P, P]
    lib.ts_search2d_workspace_bytes.argtypes = [i32, i32, i32]
    lib.ts_search2d_workspace_bytes.restype = sz
    lib.ts_threshold_search2d.argtypes = [P, i32, i32, i32, P, P, sz, P, P, P, P]
    lib.ts_open2d_workspace_bytes.argtypes = [i32, i32, i32]
    lib.ts_open2d_workspace_bytes.restype = sz
    lib.ts_open2d.argtypes = [_Batch, i32, i32, Binning, i32, P, sz, P, P, P, P]
    lib.ts_search_dp_workspace_bytes.argtypes = [i32, i32, i32, i32]
    lib.ts_search_dp_workspace_bytes.restype = sz
    lib.ts_threshold_search_dp.argtypes = [P, P, i32, i32, i32, i32, P, P, sz, P, P, P, P]
    for f in (lib.ts_histogram, lib.ts_prefix, lib.ts_threshold_search, lib.ts_threshold_search_noalloc, lib.ts_segment, lib.ts_label, lib.ts_label_sets,
              lib.ts_log2_f32, lib.ts_histogram2d, lib.ts_threshold_search2d, lib.ts_threshold_search_dp,
              lib.ts_open2d, lib.ts_issue_rate):
        f.restype = ctypes.c_int
    lib.ts_last_error.argtypes = []
    lib.ts_last_error.restype = ctypes.c_char_p
    lib.ts_abi_version.restype = ctypes.c_int32
    if lib.ts_abi_version() != ABI_VERSION:
        raise ImportError("libts ABI version mismatch")
    return lib


_lib = _load()


def _check(st: int):
    if st != TS_OK:
        raise TsError(st, _lib.ts_last_error().decode())


def _stream(stream) -> Optional[int]:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _on(stream):
    """Context in which the binding allocates the tensors of a call: the
    stream the call's kernels run on, so the caching allocator reuses that
    memory only after them (torch's current stream when none is given)."""
    return torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


_TUNED: dict = {}  # size-class key -> Tuning or None, for "auto" (the default cache is read once)


def _tune(tune, key_fn=None, lookup_fn=None):
    """None: library defaults; "auto": the autotuner's cached shapes for this
    size class (defaults if none; lookup_fn(autotune) in place of the cache
    entry of the key when given), resolved once per size class; a dict or
    Tuning: those shapes."""
    if tune is None:
        return None
    if isinstance(tune, str):
        if tune != "auto":
            raise ValueError(f"unknown tuning {tune!r}")
        if not key_fn:
            return None
        from . import autotune
        key = key_fn(autotune)
        if key not in _TUNED:
            d = lookup_fn(autotune) if lookup_fn else autotune.lookup(key)
            _TUNED[key] = Tuning.from_dict(d) if d else None
        t = _TUNED[key]
        return ctypes.byref(t) if t is not None else None
    if isinstance(tune, dict):
        tune = Tuning.from_dict(tune)
    return ctypes.byref(tune)


def device_table(values: Sequence[int], device, stream=None) -> torch.Tensor:
    """int64 device array of `values`, copied from pinned host memory without
    blocking the host, ordered on `stream` (default: the current stream)."""
    h = torch.tensor(list(values) or [0], dtype=torch.int64).pin_memory()
    with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream(device)):
        return h.to(device, non_blocking=True)


class Batch:
    """Device segment table for a batch of problems.

    ``segments`` is a list of 1-D views (int16, CUDA) -- e.g. the slices of a
    volume or whole volumes.  The table holds device pointers and the voxel
    offsets; the tensors are kept alive by this object.  The table is copied
    on `stream` (default: the current stream): use the batch on that stream,
    or synchronise first."""

    def __init__(self, segments: Sequence[torch.Tensor], device=None, stream=None):
        segs = list(segments)
        dev = device or (segs[0].device if segs else torch.device("cuda"))
        for s in segs:
            if s.dtype != torch.int16 or not s.is_cuda or not s.is_contiguous():
                raise ValueError("segments must be contiguous int16 CUDA tensors")
        self.segments = segs
        self.sizes = [int(s.numel()) for s in segs]
        offs = [0]
        for n in self.sizes:
            offs.append(offs[-1] + n)
        self.total = offs[-1]
        self.nseg = len(segs)
        self.ptrs = device_table([s.data_ptr() for s in segs], dev, stream)
        self.offs = device_table(offs, dev, stream)
        self._c = _Batch(self.ptrs.data_ptr(), self.offs.data_ptr(), self.nseg, self.total)

    @classmethod
    def slices(cls, volume: torch.Tensor, stream=None) -> "Batch":
        """One problem per slice of a (Z, H, W) volume."""
        v = volume.contiguous()
        return cls([v[z].reshape(-1) for z in range(v.shape[0])], stream=stream)

    @classmethod
    def whole(cls, volumes: Iterable[torch.Tensor]) -> "Batch":
        """One problem per volume."""
        return cls([v.contiguous().reshape(-1) for v in volumes])


def binning(lo: int, hi: int, nbins: int) -> Binning:
    return Binning(int(lo), int(hi), int(nbins))


def histogram(batch: Batch, bin: Binning, out: Optional[torch.Tensor] = None, tune=None, stream=None):
    if out is None:
        with _on(stream):
            out = torch.empty((batch.nseg, bin.nbins), dtype=torch.int32, device=batch.ptrs.device)
    t = _tune(tune, lambda a: a.key_histogram(batch.nseg, batch.total, bin.nbins))
    _check(_lib.ts_histogram(batch._c, bin, _ptr(out), t, _stream(stream)))
    return out


def _qs(q):
    """(tuple of q values, batched?) for a scalar or a sequence."""
    if isinstance(q, (int, float)):
        return (float(q),), False
    qs = tuple(float(x) for x in q)
    return qs, True


def _qarr(qs):
    return (ctypes.c_double * len(qs))(*qs) if qs else None


def prefix(hist: torch.Tensor, q, P=None, Q=None, stream=None):
    """P [nseg, L] and Q: [nseg, L] for a scalar q, [nq, nseg, L] for a sequence."""
    nseg, L = hist.shape
    qs, batched = _qs(q)
    with _on(stream):
        if P is None:
            P = torch.empty((nseg, L), dtype=torch.float64, device=hist.device)
        if Q is None:
            Q = torch.empty(((len(qs),) if batched else ()) + (nseg, L), dtype=torch.float64, device=hist.device)
    _check(_lib.ts_prefix(_ptr(hist), nseg, L, len(qs), _qarr(qs), _ptr(P), _ptr(Q), _stream(stream)))
    return P, Q


def workspace_bytes(nseg: int, nbins: int, k: int, mode: int = SEARCH_FP32_TIECHECK, nq: int = 1) -> int:
    return int(_lib.ts_search_workspace_bytes(nseg, nbins, k, nq, mode))


def threshold_search(P: torch.Tensor, Q: torch.Tensor, k: int, q, mode: int = SEARCH_FP32_TIECHECK,
                     ws: Optional[torch.Tensor] = None, out=None, tune=None, stream=None):
    """thr [.., nseg, k], obj and status [.., nseg]; the leading [nq] dimension
    is present when q is a sequence."""
    nseg, L = P.shape
    qs, batched = _qs(q)
    nq = len(qs)
    lead = (nq,) if batched else ()
    need = workspace_bytes(nseg, L, k, mode, nq)
    with _on(stream):
        if ws is None:
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=P.device)
        if out is None:
            thr = torch.empty(lead + (nseg, k), dtype=torch.int32, device=P.device)
            obj = torch.empty(lead + (nseg,), dtype=torch.float64, device=P.device)
            status = torch.empty(lead + (nseg,), dtype=torch.int32, device=P.device)
        else:
            thr, obj, status = out
    t = _tune(tune, lambda a: a.key_search(nseg * nq, L, k, mode))
    _check(_lib.ts_threshold_search(_ptr(P), _ptr(Q), nseg, L, int(k), nq, _qarr(qs), int(mode), _ptr(ws),
                                    ws.numel(), _ptr(thr), _ptr(obj), _ptr(status), t, _stream(stream)))
    return thr, obj, status


NOALLOC_SCRATCH_BYTES = 64 << 20


def threshold_search_noalloc(P: torch.Tensor, Q: torch.Tensor, k: int, q, mode: int = SEARCH_FP32_TIECHECK,
                             out=None, tune=None, stream=None):
    """threshold_search without a workspace: the library's fixed per-GPU
    scratch is used (calls that overlap on one GPU race on it).  With `out`
    (thr, obj, status) nothing is allocated here either."""
    nseg, L = P.shape
    qs, batched = _qs(q)
    nq = len(qs)
    lead = (nq,) if batched else ()
    if out is None:
        with _on(stream):
            thr = torch.empty(lead + (nseg, k), dtype=torch.int32, device=P.device)
            obj = torch.empty(lead + (nseg,), dtype=torch.float64, device=P.device)
            status = torch.empty(lead + (nseg,), dtype=torch.int32, device=P.device)
    else:
        thr, obj, status = out
    t = _tune(tune, lambda a: a.key_search(nseg * nq, L, k, mode))
    _check(_lib.ts_threshold_search_noalloc(_ptr(P), _ptr(Q), nseg, L, int(k), nq, _qarr(qs), int(mode),
                                            _ptr(thr), _ptr(obj), _ptr(status), t, _stream(stream)))
    return thr, obj, status


DP_MAX_K = 16
MORPH_MAX_RADIUS = 32


def open2d(batch: Batch, height: int, width: int, bin: Binning, radius: int = 10, ws: Optional[torch.Tensor] = None,
           opened: Optional[torch.Tensor] = None, residue: Optional[torch.Tensor] = None,
           residue16: Optional[torch.Tensor] = None, want=("opened", "residue"), stream=None):
    """Gray-scale opening of each image by a flat disk (uint8 [nseg, H, W]) and
    the residue gray - opened (uint8, and as int16 when "residue16" is
    wanted); returns (opened, residue, residue16), None for an output not
    wanted."""
    dev = batch.ptrs.device
    shape = (batch.nseg, height, width)
    need = int(_lib.ts_open2d_workspace_bytes(batch.nseg, height, width))
    with _on(stream):
        if opened is None and "opened" in want:
            opened = torch.empty(shape, dtype=torch.uint8, device=dev)
        if residue is None and "residue" in want:
            residue = torch.empty(shape, dtype=torch.uint8, device=dev)
        if residue16 is None and "residue16" in want:
            residue16 = torch.empty(shape, dtype=torch.int16, device=dev)
        if ws is None:
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)

    def p(t):
        return _ptr(t) if t is not None else None

    _check(_lib.ts_open2d(batch._c, height, width, bin, int(radius), _ptr(ws), ws.numel(), p(opened), p(residue),
                          p(residue16), _stream(stream)))
    return opened, residue, residue16


def workspace_dp_bytes(nseg: int, nbins: int, k: int, nq: int = 1) -> int:
    return int(_lib.ts_search_dp_workspace_bytes(nseg, nbins, k, nq))


def threshold_search_dp(P: torch.Tensor, Q: torch.Tensor, k: int, q, ws: Optional[torch.Tensor] = None, out=None,
                        stream=None):
    """The arg max of threshold_search by dynamic programming, k in 1..DP_MAX_K;
    outputs as for threshold_search."""
    nseg, L = P.shape
    qs, batched = _qs(q)
    nq = len(qs)
    lead = (nq,) if batched else ()
    need = workspace_dp_bytes(nseg, L, k, nq)
    with _on(stream):
        if ws is None:
            ws = torch.empty(max(need, 8), dtype=torch.uint8, device=P.device)
        if out is None:
            thr = torch.empty(lead + (nseg, k), dtype=torch.int32, device=P.device)
            obj = torch.empty(lead + (nseg,), dtype=torch.float64, device=P.device)
            status = torch.empty(lead + (nseg,), dtype=torch.int32, device=P.device)
        else:
            thr, obj, status = out
    _check(_lib.ts_threshold_search_dp(_ptr(P), _ptr(Q), nseg, L, int(k), nq, _qarr(qs), _ptr(ws), ws.numel(),
                                       _ptr(thr), _ptr(obj), _ptr(status), _stream(stream)))
    return thr, obj, status


def label(batch: Batch, bin: Binning, thr: torch.Tensor, k: int, outs: Optional[List[torch.Tensor]] = None,
          out_ptrs: Optional[torch.Tensor] = None, tune=None, stream=None):
    dev = batch.ptrs.device
    if outs is None:
        with _on(stream):
            outs = [torch.empty(n, dtype=torch.uint8, device=dev) for n in batch.sizes]
    if out_ptrs is None:
        out_ptrs = device_table([o.data_ptr() for o in outs], dev, stream)
    t = _tune(tune, lambda a: a.key_label(batch.nseg, batch.total, k))
    _check(_lib.ts_label(batch._c, bin, _ptr(thr), int(k), _ptr(out_ptrs), t, _stream(stream)))
    return outs


MAX_LABEL_SETS = 4


def label_sets(batch: Batch, bin: Binning, thrs: Sequence[torch.Tensor], k: int,
               outs: Optional[List[List[torch.Tensor]]] = None, out_ptrs: Optional[Sequence[torch.Tensor]] = None,
               tune=None, stream=None):
    """Labels for several threshold sets (each int32 [nseg, k]) in one pass."""
    dev = batch.ptrs.device
    n = len(thrs)
    if outs is None:
        with _on(stream):
            outs = [[torch.empty(m, dtype=torch.uint8, device=dev) for m in batch.sizes] for _ in range(n)]
    if out_ptrs is None:
        out_ptrs = [device_table([o.data_ptr() for o in oq], dev, stream) for oq in outs]
    thr_arr = (ctypes.c_void_p * max(n, 1))(*[t.data_ptr() for t in thrs])
    out_arr = (ctypes.c_void_p * max(n, 1))(*[p.data_ptr() for p in out_ptrs])
    t = _tune(tune, lambda a: a.key_label(batch.nseg, batch.total, k, n))
    _check(_lib.ts_label_sets(batch._c, bin, n, ctypes.cast(thr_arr, ctypes.c_void_p), int(k),
                              ctypes.cast(out_arr, ctypes.c_void_p), t, _stream(stream)))
    return outs


def segment_workspace_bytes(nseg: int, nbins: int, k: int, nq: int = 1, mode: int = SEARCH_FP32_TIECHECK,
                            labels: bool = True) -> int:
    return int(_lib.ts_segment_workspace_bytes(nseg, nbins, k, nq, mode, 1 if labels else 0))


def segment(batch: Batch, bin: Binning, k: int, q, mode: int = SEARCH_FP32_TIECHECK, labels: bool = True,
            hist=None, out=None, label_outs=None, out_ptrs=None, ws=None, tune=None, stream=None):
    """The whole path in one call (ts_segment): histograms [nseg, L], (thr,
    obj, status) as threshold_search ([nq] leading when q is a sequence) and,
    with labels, per q a list of per-problem uint8 label tensors (None when
    out_ptrs are given).  ws: a workspace of segment_workspace_bytes (any
    contents), allocated here by default."""
    qs, batched = _qs(q)
    nq, nseg, L = len(qs), batch.nseg, bin.nbins
    dev = batch.ptrs.device
    lead = (nq,) if batched else ()
    need = segment_workspace_bytes(nseg, L, k, nq, mode, labels)
    with _on(stream):
        if hist is None:
            hist = torch.empty((nseg, L), dtype=torch.int32, device=dev)
        if out is None:
            out = (torch.empty(lead + (nseg, k), dtype=torch.int32, device=dev),
                   torch.empty(lead + (nseg,), dtype=torch.float64, device=dev),
                   torch.empty(lead + (nseg,), dtype=torch.int32, device=dev))
        if ws is None:
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        if labels and out_ptrs is None:
            if label_outs is None:
                label_outs = [[torch.empty(int(n), dtype=torch.uint8, device=dev) for n in batch.sizes] for _ in qs]
            out_ptrs = [device_table([o.data_ptr() for o in oq], dev, stream) for oq in label_outs]
    thr, obj, status = out
    arr = None
    if labels:
        arr = (ctypes.c_void_p * nq)(*[p.data_ptr() for p in out_ptrs])
    t = _tune(tune, lambda a: a.key_segment(nseg, batch.total, L, k, nq),
              lambda a: a.lookup_segment(nseg, batch.total, L, k, nq, mode))
    _check(_lib.ts_segment(batch._c, bin, int(k), nq, _qarr(qs), int(mode), _ptr(hist), _ptr(thr), _ptr(obj),
                           _ptr(status), ctypes.cast(arr, ctypes.c_void_p) if labels else None, _ptr(ws),
                           ws.numel(), t, _stream(stream)))
    return hist, out, label_outs


def segment_steps(batch: Batch, bin: Binning, k: int, q: float, mode: int = SEARCH_FP32_TIECHECK, tune=None,
                  stream=None):
    """histogram -> prefix -> search -> label for every problem of the batch,
    as four separate calls."""
    h = histogram(batch, bin, tune=tune, stream=stream)
    P, Q = prefix(h, q, stream=stream)
    thr, obj, status = threshold_search(P, Q, k, q, mode, tune=tune, stream=stream)
    labels = label(batch, bin, thr, k, tune=tune, stream=stream)
    return h, (P, Q), (thr, obj, status), labels


class Segmentation:
    """Result of batch_segment: the problems' histograms, thresholds
    ([nq, nseg, k]), objectives and statuses ([nq, nseg]) and, per q, the
    label maps of every input volume in its own shape (uint8)."""

    def __init__(self, hist, thr, obj, status, labels, residues=None):
        self.hist, self.thr, self.obj, self.status, self.labels = hist, thr, obj, status, labels
        self.residues = residues  # int16 residue volumes when the opening ran first


def batch_segment(volumes: Sequence[torch.Tensor], bin: Binning, k: int, q, per: str = "slice",
                  mode: int = SEARCH_FP32_TIECHECK, method: str = "auto", open_radius: Optional[int] = None,
                  tune=None, stream=None) -> Segmentation:
    """Segment a list of int16 CUDA volumes of any shapes in one launch per
    stage: one problem per slice (per="slice") or per volume
    (per="volume"); q a value or a sequence of up to MAX_LABEL_SETS values
    (all q searched in one launch, labelled in one pass); method "exhaustive"
    (ts_threshold_search with `mode`), "dp" (ts_threshold_search_dp), "2d"
    (the two-dimensional form: per="slice", k = 1, every volume with the same
    slice shape; 2D histograms of (gray level, 3x3 average gray level), the
    arg max pair (t, s), labels from t alone; hist is then [nseg, L, L] and
    thr an [nq, nseg, 2] view holding (t, s)) or "auto" (exhaustive for
    k <= 3, dp beyond).  With open_radius (per="slice" only), each slice is
    first opened by that disk and the threshold is selected and applied on the
    residue (the paper's segmentation order; gray levels through the identity
    binning).  Only marshalling: every step runs in libts."""
    if per not in ("slice", "volume"):
        raise ValueError("per must be 'slice' or 'volume'")
    # every tensor this call makes (copies, outputs) is allocated on the
    # stream the kernels run on
    with _on(stream):
        return _batch_segment(volumes, bin, k, q, per, mode, method, open_radius, tune, stream)


def _batch_segment(volumes, bin, k, q, per, mode, method, open_radius, tune, stream) -> Segmentation:
    vols = [v.contiguous() for v in volumes]
    qs, batched = _qs(q)
    if len(qs) > MAX_LABEL_SETS:
        raise ValueError(f"at most {MAX_LABEL_SETS} q values")
    if method == "auto":
        method = "exhaustive" if k <= 3 else "dp"
    residues = None
    if open_radius is not None:
        if per != "slice":
            raise ValueError("the opening works on images: use per='slice'")
        residues = []
        for v in vols:
            if v.dim() != 3:
                raise ValueError("open_radius needs (Z, H, W) volumes")
            _, _, r16 = open2d(Batch.slices(v, stream=stream), v.shape[1], v.shape[2], bin, open_radius,
                               want=("residue16",), stream=stream)
            residues.append(r16)
        src = residues
        bin = binning(0, bin.nbins - 1, bin.nbins)
    else:
        src = vols
    if per == "slice":
        segs = [v[z].reshape(-1) for v in src for z in range(v.shape[0])]
    else:
        segs = [v.reshape(-1) for v in src]
    batch = Batch(segs, stream=stream)
    if method == "2d":
        if per != "slice" or k != 1:
            raise ValueError("the two-dimensional form takes per='slice' and k = 1")
        shapes = {tuple(v.shape[1:]) for v in src}
        if len(shapes) != 1 or any(v.dim() != 3 for v in src):
            raise ValueError("the two-dimensional form needs (Z, H, W) volumes of one slice shape")
        (Hh, Ww), = shapes
        h = histogram2d(batch, Hh, Ww, bin, stream=stream)
        thr2, obj, status = threshold_search2d(h, list(qs), stream=stream)  # [nq, 2, nseg]
        labels = [[torch.empty(v.shape, dtype=torch.uint8, device=v.device) for v in src] for _ in qs]
        outs = [[lv[z].reshape(-1) for lv in lj for z in range(lv.shape[0])] for lj in labels]
        label_sets(batch, bin, [thr2[j, 0] for j in range(len(qs))], 1, outs=outs, tune=tune, stream=stream)
        return Segmentation(h, thr2.transpose(1, 2), obj, status, labels, residues)
    h = histogram(batch, bin, tune=tune, stream=stream)
    P, Q = prefix(h, list(qs), stream=stream)
    if method == "dp":
        thr, obj, status = threshold_search_dp(P, Q, k, list(qs), stream=stream)
    else:
        thr, obj, status = threshold_search(P, Q, k, list(qs), mode, tune=tune, stream=stream)
    # label maps in each volume's shape; the label pass writes every problem
    # straight into its slice (or volume) of them
    labels = [[torch.empty(v.shape, dtype=torch.uint8, device=v.device) for v in src] for _ in qs]
    if per == "slice":
        outs = [[lv[z].reshape(-1) for lv in lj for z in range(lv.shape[0])] for lj in labels]
    else:
        outs = [[lv.reshape(-1) for lv in lj] for lj in labels]
    label_sets(batch, bin, [thr[j] for j in range(len(qs))], k, outs=outs, tune=tune, stream=stream)
    return Segmentation(h, thr, obj, status, labels, residues)


def log2_f32(x: torch.Tensor, stream=None) -> torch.Tensor:
    """The FP32 base-2 logarithm the search keys use (diagnostic)."""
    if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous float32 CUDA tensor")
    with _on(stream):
        y = torch.empty_like(x)
    _check(_lib.ts_log2_f32(_ptr(x), _ptr(y), x.numel(), _stream(stream)))
    return y


def issue_rate(op: int, blocks: int, iters: int, out: torch.Tensor, stream=None) -> None:
    """One launch of the issue-rate probe (diagnostic): op 0 plain FP32 adds,
    1 v_log_f32, 2 the search's class-term mix; out: float32 [blocks * 256]."""
    if out.dtype != torch.float32 or not out.is_cuda or out.numel() < blocks * 256:
        raise ValueError("out must be a float32 CUDA tensor of at least blocks * 256 elements")
    _check(_lib.ts_issue_rate(op, blocks, iters, _ptr(out), _stream(stream)))


def histogram2d(batch: Batch, height: int, width: int, bin: Binning, out: Optional[torch.Tensor] = None,
                stream=None) -> torch.Tensor:
    """2D histograms uint32 [nseg, L, L] (int32 storage) of height x width images."""
    L = bin.nbins
    if out is None:
        with _on(stream):
            out = torch.empty((batch.nseg, L, L), dtype=torch.int32, device=batch.ptrs.device)
    _check(_lib.ts_histogram2d(batch._c, int(height), int(width), bin, _ptr(out), _stream(stream)))
    return out


def workspace2d_bytes(nseg: int, nbins: int, nq: int = 1) -> int:
    return int(_lib.ts_search2d_workspace_bytes(nseg, nbins, nq))


def threshold_search2d(hist2d: torch.Tensor, q, ws: Optional[torch.Tensor] = None, out=None, stream=None):
    """thresholds int32 [.., 2, nseg] (row 0: t, row 1: s), objectives and
    statuses [.., nseg]; the leading [nq] dimension is present when q is a
    sequence.  Row 0 is the k = 1 threshold array of `label`."""
    nseg, L, _ = hist2d.shape
    qs, batched = _qs(q)
    nq = len(qs)
    lead = (nq,) if batched else ()
    need = workspace2d_bytes(nseg, L, nq)
    with _on(stream):
        if ws is None:
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=hist2d.device)
        if out is None:
            thr = torch.empty(lead + (2, nseg), dtype=torch.int32, device=hist2d.device)
            obj = torch.empty(lead + (nseg,), dtype=torch.float64, device=hist2d.device)
            status = torch.empty(lead + (nseg,), dtype=torch.int32, device=hist2d.device)
        else:
            thr, obj, status = out
    _check(_lib.ts_threshold_search2d(_ptr(hist2d), nseg, L, nq, _qarr(qs), _ptr(ws), ws.numel(), _ptr(thr),
                                      _ptr(obj), _ptr(status), _stream(stream)))
    return thr, obj, status


def last_error() -> str:
    return _lib.ts_last_error().decode()
