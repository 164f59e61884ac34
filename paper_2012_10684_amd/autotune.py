"""Launch-shape autotuner for libts.

Every kernel of the path has launch-shape knobs (``ts_tuning``): histogram
workgroup size, LDS replicas and persistent workgroups per CU; label workgroup
size and vectors per thread; search columns per lane, rows per tile, path (one
workgroup per problem or one launch per phase) and workgroup size.  No knob
changes any output bit, so the tuner may pick any of them on speed alone.

``Autotuner`` times each candidate on the caller's own inputs (median of HIP
event timings on the launch stream, after warm-up) and stores the fastest per
key in a JSON cache.  A key is (GPU architecture, kernel, size class), where
size classes are powers of two of the problem count and voxel count, the bin
count, k and the search mode.  ``lookup`` returns the cached tuning for a key
or None (library defaults).  The cache file is ``TS_AUTOTUNE_CACHE`` if set,
else ``tuned.json`` next to this file (shapes measured on MI355X).

Command line: ``python -m paper_2012_10684_amd.autotune --workload NAME
[--out FILE]`` tunes one of the built-in workloads and writes the cache.
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import statistics
import sys
from typing import Callable, Dict, Iterable, Optional

import torch

from . import api

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(_HERE, "tuned.json")


def cache_path() -> str:
    return os.environ.get("TS_AUTOTUNE_CACHE", DEFAULT_CACHE)


_ARCH: Dict[int, str] = {}


def _arch() -> str:
    """Architecture name of the current device (memoised per device)."""
    try:
        i = torch.cuda.current_device()
    except Exception:  # no GPU: keys still work for reading the cache
        return "gfx950"
    a = _ARCH.get(i)
    if a is None:
        try:
            a = torch.cuda.get_device_properties(i).gcnArchName.split(":")[0]
        except Exception:
            a = "gfx950"
        _ARCH[i] = a
    return a


def _p2(n: int) -> int:
    return 0 if n <= 0 else int(math.ceil(math.log2(n)))


def key_histogram(nseg: int, total: int, L: int) -> str:
    return f"{_arch()}|histogram|L={L}|nseg=2^{_p2(nseg)}|vox=2^{_p2(total)}"


def key_label(nseg: int, total: int, k: int, nsets: int = 1) -> str:
    sets = "" if nsets == 1 else f"|sets={nsets}"
    return f"{_arch()}|label|k={k}{sets}|nseg=2^{_p2(nseg)}|vox=2^{_p2(total)}"


def key_search(nseg: int, L: int, k: int, mode: int) -> str:
    return f"{_arch()}|search|L={L}|k={k}|mode={mode}|nseg=2^{_p2(nseg)}"


def key_segment(nseg: int, total: int, L: int, k: int, nq: int) -> str:
    return f"{_arch()}|segment|L={L}|k={k}|nq={nq}|nseg=2^{_p2(nseg)}|vox=2^{_p2(total)}"


def histogram_space(L: int) -> Iterable[dict]:
    # min_chunk bounds the workgroup count from below in voxels per workgroup:
    # large chunks pay off when each workgroup flushes many bins
    for r, b, w, m in itertools.product((1, 2, 4, 8, 16, 32), (256, 512, 1024), (1, 2, 4, 8), (0, 32768, 131072)):
        if L * r * 4 <= 160 * 1024 and w * L * r * 4 <= 160 * 1024 and L * r >= 1024:
            d = dict(hist_replicas=r, hist_block=b, hist_wg_per_cu=w)
            if m:
                d["min_chunk"] = m
            yield d


def label_space() -> Iterable[dict]:
    for b, u in itertools.product((64, 128, 256, 512, 1024), (1, 2, 4)):
        yield dict(label_block=b, label_vecs=u)


def search_space(L: int, k: int) -> Iterable[dict]:
    for c, r in itertools.product((1, 2, 4), (16, 32, 64)):
        if k == 3 and r != 16:
            continue  # rows per tile only shape k = 2 tiles
        yield dict(search_cols=c, search_rows=r, search_path=2)
        if k == 1 or (k == 2 and L <= 1024):
            for tb in (256, 512, 1024):
                yield dict(search_cols=c, search_rows=r, search_path=1, search_block=tb)


def time_call(fn: Callable[[], None], reps: int = 10, warmup: int = 3, stream=None) -> float:
    """Median duration (s) of fn() measured with events on the launch stream."""
    s = stream or torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        b.synchronize()
        times.append(a.elapsed_time(b) * 1e-3)
    return statistics.median(times)


class Autotuner:
    def __init__(self, path: Optional[str] = None, verbose: bool = False):
        self.path = path or cache_path()
        self.verbose = verbose
        self.cache: Dict[str, dict] = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                self.cache = json.load(f)

    def save(self, path: Optional[str] = None):
        p = path or self.path
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.cache, f, indent=1, sort_keys=True)
        os.replace(tmp, p)

    def lookup(self, key: str) -> Optional[dict]:
        e = self.cache.get(key)
        return dict(e["tuning"]) if e else None

    def _sweep(self, key: str, space: Iterable[dict], run: Callable[[dict], None], reps: int) -> dict:
        best, best_t, tried = None, float("inf"), []
        base_t = time_call(lambda: run({}), reps)
        for cand in space:
            try:
                t = time_call(lambda: run(cand), reps)
            except api.TsError:
                continue
            tried.append((t, cand))
            if t < best_t:
                best, best_t = cand, t
        if best is None or base_t <= best_t:
            best, best_t = {}, base_t
        self.cache[key] = {"tuning": best, "us": round(best_t * 1e6, 3), "default_us": round(base_t * 1e6, 3),
                           "candidates": len(tried)}
        if self.verbose:
            print(f"{key}: {best} {best_t * 1e6:.2f} us (default {base_t * 1e6:.2f} us, {len(tried)} tried)",
                  flush=True)
        return best

    def tune_histogram(self, batch: api.Batch, binn: api.Binning, out: torch.Tensor, reps: int = 10) -> dict:
        key = key_histogram(batch.nseg, batch.total, binn.nbins)
        return self._sweep(key, histogram_space(binn.nbins),
                           lambda t: api.histogram(batch, binn, out=out, tune=t or None), reps)

    def tune_label(self, batch: api.Batch, binn: api.Binning, thr: torch.Tensor, k: int, outs, optrs,
                   reps: int = 10) -> dict:
        key = key_label(batch.nseg, batch.total, k)
        return self._sweep(key, label_space(),
                           lambda t: api.label(batch, binn, thr, k, outs=outs, out_ptrs=optrs, tune=t or None), reps)

    def tune_label_sets(self, batch: api.Batch, binn: api.Binning, thrs, k: int, outs, optrs,
                        reps: int = 10) -> dict:
        key = key_label(batch.nseg, batch.total, k, len(thrs))
        return self._sweep(key, label_space(),
                           lambda t: api.label_sets(batch, binn, thrs, k, outs=outs, out_ptrs=optrs,
                                                    tune=t or None), reps)

    def tune_search(self, P: torch.Tensor, Q: torch.Tensor, k: int, q, mode: int, ws: torch.Tensor, out,
                    reps: int = 10) -> dict:
        """q: one value, or a sequence searched in one launch (key over nq x nseg problems)."""
        nseg, L = P.shape
        nq = 1 if isinstance(q, (int, float)) else len(q)
        key = key_search(nseg * nq, L, k, mode)
        return self._sweep(key, search_space(L, k),
                           lambda t: api.threshold_search(P, Q, k, q, mode, ws=ws, out=out, tune=t or None), reps)


_default: Optional[Autotuner] = None


def lookup(key: str) -> Optional[dict]:
    """Cached tuning for a key from the default cache, or None."""
    global _default
    if _default is None:
        _default = Autotuner()
    return _default.lookup(key)


def lookup_segment(nseg: int, total: int, L: int, k: int, nq: int, mode: int) -> Optional[dict]:
    """Tuning of a ts_segment call: its own cache entry if there is one, else
    the entries of the separate steps it may run (histogram, search of nseg x
    nq problems, labels of nq sets), whose fields do not overlap; None if none
    is cached."""
    own = lookup(key_segment(nseg, total, L, k, nq))
    if own is not None:
        return own
    merged = {}
    for key in (key_histogram(nseg, total, L), key_search(nseg * nq, L, k, mode), key_label(nseg, total, k, nq)):
        merged.update(lookup(key) or {})
    return merged or None


# ---------------------------------------------------------------------------- CLI

def _tune_workload(name: str, tuner: Autotuner):
    from . import synth

    dev = torch.device("cuda:0")
    if name == "volume300":
        vol, per_slice, lo, hi, L, k, qs = synth.workload_volume300(0), True, -1024, -200, 256, 2, (0.5, 0.8, 1.5)
    elif name == "volume600":
        vol, per_slice, lo, hi, L, k, qs = synth.workload_volume600(0), False, -1024, 3071, 1024, 3, (0.8,)
    elif name == "slice":
        vol, per_slice, lo, hi, L, k, qs = synth.workload_slice(0)[None], False, -1024, 3071, 4096, 1, (0.8,)
    elif name == "serving":
        vol, per_slice, lo, hi, L, k, qs = synth.serving_volume(0, 300, 512), False, -1024, 3071, 512, 3, (0.8,)
    else:
        raise SystemExit(f"unknown workload {name}")
    dv = torch.from_numpy(vol).to(dev)
    batch = api.Batch.slices(dv) if per_slice else api.Batch([dv.reshape(-1)])
    binn = api.binning(lo, hi, L)
    hist = api.histogram(batch, binn)
    tuner.tune_histogram(batch, binn, hist)
    # every q of the workload in one search launch, as the benchmark runs it
    nq = len(qs)
    P, Q = api.prefix(hist, qs)
    ws = torch.empty(api.workspace_bytes(batch.nseg, L, k, api.SEARCH_FP32_TIECHECK, nq), dtype=torch.uint8,
                     device=dev)
    out = (torch.empty((nq, batch.nseg, k), dtype=torch.int32, device=dev),
           torch.empty((nq, batch.nseg), dtype=torch.float64, device=dev),
           torch.empty((nq, batch.nseg), dtype=torch.int32, device=dev))
    tuner.tune_search(P, Q, k, qs, api.SEARCH_FP32_TIECHECK, ws, out)
    thrs = [out[0][j] for j in range(nq)]
    outs = [[torch.empty(n, dtype=torch.uint8, device=dev) for n in batch.sizes] for _ in thrs]
    optrs = [torch.tensor([o.data_ptr() for o in oq], dtype=torch.int64).to(dev) for oq in outs]
    tuner.tune_label(batch, binn, thrs[0], k, outs[0], optrs[0])
    if len(thrs) > 1:
        tuner.tune_label_sets(batch, binn, thrs, k, outs, optrs)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", action="append", required=True,
                    help="volume300 | volume600 | slice | serving (repeatable)")
    ap.add_argument("--out", default=None, help="cache file to write (default: the cache in use)")
    args = ap.parse_args(argv)
    tuner = Autotuner(path=args.out or cache_path(), verbose=True)
    for w in args.workload:
        print(f"== tuning {w}", flush=True)
        _tune_workload(w, tuner)
        tuner.save()
    print(f"wrote {tuner.path}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
