"""Continuous-batching serving of segmentation requests on one GPU.

A request is one int16 volume (one problem: whole-volume histogram, k
thresholds for each entropic index q, one label map per q).  Requests queue in
arrival order; the scheduler admits the requests that have arrived, in order,
while the batch fits a voxel budget, a request cap, and the device memory that
is free right now (and an optional fixed budget of device bytes in flight).
Each admitted batch runs as

    H2D stream:      pinned host volumes -> device
    compute stream:  ts_histogram -> ts_prefix (all q) -> ts_threshold_search
                     (all q, one launch) -> ts_label_sets
    D2H stream:      label maps -> pinned host buffers from a pool

with events between the streams, so the upload of batch i+1 overlaps the
compute of batch i and the download of batch i-1 (all streams at the default
priority).  A request's histogram and thresholds stay resident with its batch
until the download completes, so every q of the request shares one histogram
pass.  Latency is measured from the request's arrival to its labels being in
host memory; the device time of its batch (upload start to download end, and
the kernels alone) is measured with events.

A request that cannot be served (not an int16 volume, larger than any budget,
or a batch whose launch raises) gets a Result with `error` set; the other
requests of its batch are retried alone and the loop continues.

``Scheduler`` (admission policy and statistics) is plain Python; ``Engine``
runs the loop over a backend: ``GpuBackend`` executes batches through the HIP
library (``api``) and has no other compute path.  A backend provides
``launch(reqs) -> handle``, ``ready(handle)``, ``wait(handle)``,
``collect(handle) -> [dict per request]``, ``free_bytes()`` and
``release(result)``.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Deque, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    volume: object          # torch int16 CPU tensor (pinned for overlapped copies) or numpy array
    arrival: float          # seconds on the engine clock
    nvox: int = 0

    def __post_init__(self):
        if not self.nvox:
            self.nvox = int(np.prod(tuple(self.volume.shape)))


@dataclasses.dataclass
class Result:
    rid: int
    thr: Optional[np.ndarray]      # int32 [nq, k]
    obj: Optional[np.ndarray]      # float64 [nq]
    status: Optional[np.ndarray]   # int32 [nq]
    labels: list                   # nq host uint8 tensors (pinned), voxel order of the request
    arrival: float
    admitted: float
    done: float
    nvox: int = 0
    error: Optional[str] = None    # set when the request could not be served
    device_s: float = math.nan     # its batch on the device: upload start to download end
    kernels_s: float = math.nan    # its batch's kernels (histogram start to labels end)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Scheduler:
    """FIFO admission under a voxel budget per batch, a request cap per batch,
    the device bytes free at admission time and an optional fixed budget of
    device bytes in flight."""

    def __init__(self, bytes_per_voxel: float, hbm_budget: Optional[int], max_batch_voxels: int,
                 max_batch_requests: int = 64):
        if bytes_per_voxel <= 0 or (hbm_budget is not None and hbm_budget <= 0) or max_batch_voxels <= 0 or \
                max_batch_requests <= 0:
            raise ValueError("budgets must be positive")
        self.bpv = bytes_per_voxel
        self.hbm_budget = None if hbm_budget is None else int(hbm_budget)
        self.max_batch_voxels = int(max_batch_voxels)
        self.max_batch_requests = int(max_batch_requests)
        self.queue: Deque[Request] = collections.deque()
        self.inflight_bytes = 0

    def cost(self, r: Request) -> int:
        return int(math.ceil(r.nvox * self.bpv))

    def submit(self, r: Request):
        if self.hbm_budget is not None and self.cost(r) > self.hbm_budget:
            raise ValueError(f"request {r.rid} needs {self.cost(r)} device bytes, over the budget {self.hbm_budget}")
        if self.queue and r.arrival < self.queue[-1].arrival:
            raise ValueError("requests must be submitted in arrival order")
        self.queue.append(r)

    def admit(self, now: float, free_bytes: Optional[int] = None) -> List[Request]:
        """Requests that have arrived by `now`, in order, while they fit.  A
        request larger than the voxel budget is admitted alone.  free_bytes:
        device bytes free right now (requests in flight already hold theirs);
        the requests admitted here must fit in it together."""
        out: List[Request] = []
        vox = 0
        taken = 0
        while self.queue and self.queue[0].arrival <= now and len(out) < self.max_batch_requests:
            r = self.queue[0]
            c = self.cost(r)
            if self.hbm_budget is not None and self.inflight_bytes + c > self.hbm_budget:
                break
            if free_bytes is not None and taken + c > free_bytes:
                break
            if out and vox + r.nvox > self.max_batch_voxels:
                break
            self.queue.popleft()
            out.append(r)
            vox += r.nvox
            taken += c
            self.inflight_bytes += c
        return out

    def release(self, reqs: Sequence[Request]):
        for r in reqs:
            self.inflight_bytes -= self.cost(r)
        assert self.inflight_bytes >= 0

    def next_arrival(self) -> Optional[float]:
        return self.queue[0].arrival if self.queue else None


def latency_stats(results: Sequence[Result], wall: Optional[float] = None) -> Dict[str, float]:
    """p50 / p99 / mean / max latency (s) of the served requests, the same
    for their batches' device time, and voxel throughput."""
    served = [r for r in results if r.error is None]
    if not served:
        return {"n": 0, "errors": len(results)}
    lat = np.array([r.latency for r in served])
    d = {"n": len(served), "errors": len(results) - len(served), "p50_s": float(np.percentile(lat, 50)),
         "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()), "max_s": float(lat.max())}
    dev = np.array([r.device_s for r in served])
    if np.isfinite(dev).all():
        d.update(device_p50_s=float(np.percentile(dev, 50)), device_p99_s=float(np.percentile(dev, 99)))
    ker = np.array([r.kernels_s for r in served])
    if np.isfinite(ker).all():
        d.update(kernels_p50_s=float(np.percentile(ker, 50)), kernels_p99_s=float(np.percentile(ker, 99)))
    if wall:
        d["voxels_per_s"] = float(sum(r.nvox for r in served) / wall)
    return d


class PinnedPool:
    """Host buffers for label downloads, allocated before serving starts:
    `slots` buffers of `slot_bytes` each.  take(n) hands out a free buffer
    (its first n bytes); give(buf) returns it.  When every slot is out, take
    allocates a fresh buffer (counted in `extra`), so a caller that keeps its
    results never stalls the loop."""

    def __init__(self, slots: int, slot_bytes: int, alloc: Callable[[int], object]):
        self.alloc = alloc
        self.slot_bytes = int(slot_bytes)
        self.free = [alloc(self.slot_bytes) for _ in range(slots)]
        self.owner = {}  # id(view) -> slot buffer
        self.extra = 0

    def take(self, n: int):
        if n <= self.slot_bytes and self.free:
            buf = self.free.pop()
            view = buf[:n]
            self.owner[id(view)] = buf
            return view
        self.extra += 1
        return self.alloc(n)

    def give(self, view):
        buf = self.owner.pop(id(view), None)
        if buf is not None:
            self.free.append(buf)


class GpuBackend:
    """Runs batches on one GPU through libts on three streams (see module doc)."""

    def __init__(self, binning, k: int, qs: Sequence[float], device=None, tune="auto",
                 max_request_voxels: int = 0, pool_slots: int = 0, reserve_bytes: int = 2 << 30):
        import torch

        from . import api

        self.torch, self.api = torch, api
        self.dev = torch.device(device or "cuda:0")
        self.binn = binning
        self.k = int(k)
        self.qs = tuple(float(q) for q in qs)
        self.nq = len(self.qs)
        self.tune = tune
        self.reserve = int(reserve_bytes)
        self.s_h2d = torch.cuda.Stream(device=self.dev)
        self.s_cmp = torch.cuda.Stream(device=self.dev)
        self.s_d2h = torch.cuda.Stream(device=self.dev)
        pin = lambda n: torch.empty(n, dtype=torch.uint8, pin_memory=True)  # noqa: E731
        self.pool = PinnedPool(pool_slots, max_request_voxels, pin)
        # thresholds, objectives and statuses of one batch (64 requests x 4 q fit in 16 KiB)
        self.small_pool = PinnedPool(8, 16 << 10, pin)

    def free_bytes(self) -> int:
        """Device bytes free for new requests: what the device reports free,
        plus what the caching allocator holds unused, minus a reserve for
        the batch's small tensors and the library's workspaces."""
        torch = self.torch
        free, _ = torch.cuda.mem_get_info(self.dev)
        cached = torch.cuda.memory_reserved(self.dev) - torch.cuda.memory_allocated(self.dev)
        return max(0, int(free + cached - self.reserve))

    def launch(self, reqs: List[Request]) -> dict:
        torch, api = self.torch, self.api
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        dvols = []
        with torch.cuda.stream(self.s_h2d):
            ev[0].record(self.s_h2d)
            for r in reqs:
                v = r.volume if isinstance(r.volume, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(r.volume))
                if v.dtype != torch.int16:
                    raise TypeError(f"request {r.rid}: volume must be int16, not {v.dtype}")
                d = torch.empty(r.nvox, dtype=torch.int16, device=self.dev)
                d.copy_(v.reshape(-1), non_blocking=True)
                dvols.append(d)
        up = torch.cuda.Event()
        up.record(self.s_h2d)
        n = len(reqs)
        with torch.cuda.stream(self.s_cmp):
            self.s_cmp.wait_event(up)
            ev[1].record(self.s_cmp)
            batch = api.Batch(dvols, device=self.dev, stream=self.s_cmp)
            hist = api.histogram(batch, self.binn, tune=self.tune, stream=self.s_cmp)
            P, Q = api.prefix(hist, self.qs, stream=self.s_cmp)
            thr, obj, st = api.threshold_search(P, Q, self.k, self.qs, tune=self.tune, stream=self.s_cmp)
            outs = api.label_sets(batch, self.binn, [thr[j] for j in range(self.nq)], self.k, tune=self.tune,
                                  stream=self.s_cmp)
            ev[2].record(self.s_cmp)
        done_cmp = torch.cuda.Event()
        done_cmp.record(self.s_cmp)
        host = []
        with torch.cuda.stream(self.s_d2h):
            self.s_d2h.wait_event(done_cmp)
            for i in range(n):
                row = []
                for j in range(self.nq):
                    h = self.pool.take(reqs[i].nvox)
                    h.copy_(outs[j][i], non_blocking=True)
                    row.append(h)
                host.append(row)
            # one pinned block: objectives (8-byte aligned first), thresholds, statuses
            no, nt = obj.numel() * 8, thr.numel() * 4
            blk = self.small_pool.take(no + nt + st.numel() * 4)
            small = (blk[:no].view(torch.float64).view(obj.shape), blk[no:no + nt].view(torch.int32).view(thr.shape),
                     blk[no + nt:].view(torch.int32).view(st.shape))
            for h, d in zip(small, (obj, thr, st)):
                h.copy_(d, non_blocking=True)
            ev[3].record(self.s_d2h)
        # device tensors stay referenced until the download completes
        return dict(reqs=reqs, ev=ev, keep=(dvols, batch, hist, P, Q, thr, obj, st, outs), host=host, small=small,
                    blk=blk)

    def ready(self, b: dict) -> bool:
        return b["ev"][3].query()

    def wait(self, b: dict):
        b["ev"][3].synchronize()

    def collect(self, b: dict) -> List[dict]:
        obj, thr, st = (t.numpy().copy() for t in b["small"])  # [nq, n], [nq, n, k], [nq, n]
        self.small_pool.give(b["blk"])
        n = len(b["reqs"])
        ev = b["ev"]
        dev_s = ev[0].elapsed_time(ev[3]) * 1e-3
        ker_s = ev[1].elapsed_time(ev[2]) * 1e-3
        return [dict(thr=thr[:, i, :].copy(), obj=obj[:, i].copy(), status=st[:, i].copy(), labels=b["host"][i],
                     device_s=dev_s, kernels_s=ker_s) for i in range(n)]

    def release(self, res: Result):
        """Return a result's label buffers to the pool (after the caller is
        done with them)."""
        for t in res.labels or ():
            self.pool.give(t)
        res.labels = []


class Engine:
    """The serving loop over a backend (default: GpuBackend on one GPU)."""

    def __init__(self, binning=None, k: int = 3, qs: Sequence[float] = (0.8,), hbm_budget: Optional[int] = None,
                 max_batch_voxels: int = 1 << 30, max_batch_requests: int = 64, max_inflight: int = 2,
                 device=None, tune="auto", backend=None, max_request_voxels: int = 0, pool_slots: int = 0,
                 reserve_bytes: int = 2 << 30):
        self.qs = tuple(float(q) for q in qs)
        self.nq = len(self.qs)
        if not 1 <= self.nq <= 4:
            raise ValueError("1..4 q values per engine (one label map each, written in one pass)")
        self.k = int(k)
        self.max_inflight = max_inflight
        self.backend = backend or GpuBackend(binning, k, self.qs, device, tune, max_request_voxels, pool_slots,
                                             reserve_bytes)
        # device bytes per voxel: int16 voxels + one uint8 label per q
        self.sched = Scheduler(2 + self.nq, hbm_budget, max_batch_voxels, max_batch_requests)
        self.inflight: Deque[dict] = collections.deque()
        self.t0 = time.perf_counter()
        self.refused = 0

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def _error(self, r: Request, msg: str, admitted: float, results: List[Result]):
        results.append(Result(r.rid, None, None, None, [], r.arrival, admitted, self.now(), r.nvox, error=msg))

    def submit(self, r: Request, results: List[Result]):
        """Queue a request, or answer it with an error if it can never be
        served (not an int16 volume, or over the fixed budget)."""
        dt = getattr(r.volume, "dtype", None)
        if str(dt) not in ("int16", "torch.int16"):
            self._error(r, f"volume must be int16, not {dt}", self.now(), results)
            return
        try:
            self.sched.submit(r)
        except ValueError as e:
            self._error(r, str(e), self.now(), results)

    def _launch(self, reqs: List[Request], results: List[Result]):
        """Launch a batch; if that raises, launch its requests one by one so
        that only the failing ones get errors."""
        t_adm = self.now()
        try:
            self.inflight.append(dict(h=self.backend.launch(reqs), reqs=reqs, t_adm=t_adm))
            return
        except Exception as e:  # noqa: BLE001 -- isolate the failing request
            if len(reqs) == 1:
                self.sched.release(reqs)
                self._error(reqs[0], f"{type(e).__name__}: {e}", t_adm, results)
                return
        for r in reqs:
            self._launch([r], results)

    def _retire(self, b: dict, results: List[Result]):
        try:
            outs = self.backend.collect(b["h"])
        except Exception as e:  # noqa: BLE001
            outs = [e] * len(b["reqs"])
        t = self.now()
        for r, o in zip(b["reqs"], outs):
            if isinstance(o, Exception):
                results.append(Result(r.rid, None, None, None, [], r.arrival, b["t_adm"], t, r.nvox,
                                      error=f"{type(o).__name__}: {o}"))
            else:
                results.append(Result(r.rid, o["thr"], o["obj"], o["status"], o["labels"], r.arrival, b["t_adm"], t,
                                      r.nvox, device_s=o.get("device_s", math.nan),
                                      kernels_s=o.get("kernels_s", math.nan)))
        self.sched.release(b["reqs"])

    def poll(self, results: List[Result], block: bool = False) -> int:
        """Retire finished batches (the oldest first); returns how many."""
        n = 0
        while self.inflight:
            b = self.inflight[0]
            if block:
                self.backend.wait(b["h"])
            elif not self.backend.ready(b["h"]):
                break
            self.inflight.popleft()
            self._retire(b, results)
            n += 1
            block = False
        return n

    def release(self, res: Result):
        self.backend.release(res)

    def run(self, requests: Sequence[Request], realtime: bool = True,
            on_result: Optional[Callable[[Result], None]] = None) -> List[Result]:
        """Serve requests (arrival times on the engine clock, which starts
        now).  realtime=False makes every request arrive at once.  on_result,
        if given, sees each result as it is retired (and may release its
        buffers)."""
        self.t0 = time.perf_counter()
        results: List[Result] = []
        for r in sorted(requests, key=lambda r: r.arrival):
            if not realtime:
                r.arrival = 0.0
            self.submit(r, results)
        seen = 0

        def deliver():
            nonlocal seen
            if on_result:
                for r in results[seen:]:
                    on_result(r)
            seen = len(results)

        while self.sched.queue or self.inflight:
            self.poll(results)
            deliver()
            if len(self.inflight) < self.max_inflight:
                nxt = self.sched.next_arrival()
                if nxt is not None and nxt <= self.now():
                    reqs = self.sched.admit(self.now(), self.backend.free_bytes())
                    if reqs:
                        self._launch(reqs, results)
                        deliver()
                        continue
                    if not self.inflight:
                        # nothing holds device memory and the head still does not fit: refuse it
                        r = self.sched.queue.popleft()
                        self.refused += 1
                        self._error(r, f"request {r.rid} needs {self.sched.cost(r)} device bytes, more than are "
                                       f"free", self.now(), results)
                        deliver()
                        continue
            nxt = self.sched.next_arrival()
            now = self.now()
            if self.inflight:
                if nxt is not None and nxt > now and len(self.inflight) < self.max_inflight:
                    time.sleep(min(1e-4, nxt - now))  # an arrival may come before the oldest batch ends
                else:
                    self.poll(results, block=True)  # frees a slot and its device memory
                    deliver()
            elif nxt is None:
                break
            elif nxt > now:
                time.sleep(min(1e-3, nxt - now))
        deliver()
        return results
