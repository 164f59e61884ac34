"""Continuous-batching serving of segmentation requests on one GPU.

A request is one int16 volume (one problem: whole-volume histogram, k
thresholds for each entropic index q, one label map per q).  Requests queue in
arrival order; the scheduler admits the requests that have arrived, in order,
while the batch fits a voxel budget and the device bytes in flight fit an HBM
budget.  Each admitted batch runs as

    H2D stream:      pinned host volumes -> device
    compute stream:  ts_histogram -> ts_prefix (all q) -> ts_threshold_search
                     (all q, one launch) -> ts_label_sets
    D2H stream:      label maps -> pinned host buffers

with events between the streams, so the upload of batch i+1 overlaps the
compute of batch i and the download of batch i-1 (all streams at the default
priority).  A request's histogram and thresholds stay resident with its batch
until the download completes, so every q of the request shares one histogram
pass.  Latency is measured from the request's arrival to its labels being in
host memory.

``Scheduler`` (admission policy and statistics) is plain Python; ``Engine``
executes batches through the HIP library (``api``) and has no other compute
path.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Deque, Dict, List, Optional, Sequence

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
    thr: np.ndarray          # int32 [nq, k]
    obj: np.ndarray          # float64 [nq]
    status: np.ndarray       # int32 [nq]
    labels: list             # nq host uint8 tensors (pinned), voxel order of the request
    arrival: float
    admitted: float
    done: float
    nvox: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Scheduler:
    """FIFO admission under a voxel budget per batch, a request cap per batch
    and a budget of device bytes in flight."""

    def __init__(self, bytes_per_voxel: float, hbm_budget: int, max_batch_voxels: int, max_batch_requests: int = 64):
        if bytes_per_voxel <= 0 or hbm_budget <= 0 or max_batch_voxels <= 0 or max_batch_requests <= 0:
            raise ValueError("budgets must be positive")
        self.bpv = bytes_per_voxel
        self.hbm_budget = int(hbm_budget)
        self.max_batch_voxels = int(max_batch_voxels)
        self.max_batch_requests = int(max_batch_requests)
        self.queue: Deque[Request] = collections.deque()
        self.inflight_bytes = 0

    def cost(self, r: Request) -> int:
        return int(math.ceil(r.nvox * self.bpv))

    def submit(self, r: Request):
        if self.cost(r) > self.hbm_budget:
            raise ValueError(f"request {r.rid} needs {self.cost(r)} device bytes, over the budget {self.hbm_budget}")
        if self.queue and r.arrival < self.queue[-1].arrival:
            raise ValueError("requests must be submitted in arrival order")
        self.queue.append(r)

    def admit(self, now: float) -> List[Request]:
        """Requests that have arrived by `now`, in order, while they fit.  A
        request larger than the voxel budget is admitted alone."""
        out: List[Request] = []
        vox = 0
        while self.queue and self.queue[0].arrival <= now and len(out) < self.max_batch_requests:
            r = self.queue[0]
            c = self.cost(r)
            if self.inflight_bytes + c > self.hbm_budget:
                break
            if out and vox + r.nvox > self.max_batch_voxels:
                break
            self.queue.popleft()
            out.append(r)
            vox += r.nvox
            self.inflight_bytes += c
        return out

    def release(self, reqs: Sequence[Request]):
        for r in reqs:
            self.inflight_bytes -= self.cost(r)
        assert self.inflight_bytes >= 0

    def next_arrival(self) -> Optional[float]:
        return self.queue[0].arrival if self.queue else None


def latency_stats(results: Sequence[Result], wall: Optional[float] = None) -> Dict[str, float]:
    """p50 / p99 / mean / max latency (s) and voxel throughput."""
    if not results:
        return {"n": 0}
    lat = np.array([r.latency for r in results])
    d = {"n": len(results), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
         "mean_s": float(lat.mean()), "max_s": float(lat.max())}
    if wall:
        d["voxels_per_s"] = float(sum(r.nvox for r in results) / wall)
    return d


class Engine:
    """Runs admitted batches on one GPU through libts (see module doc)."""

    def __init__(self, binning, k: int, qs: Sequence[float], hbm_budget: int = 64 << 30,
                 max_batch_voxels: int = 1 << 30, max_batch_requests: int = 64, max_inflight: int = 2,
                 device=None, tune="auto"):
        import torch

        from . import api

        self.torch, self.api = torch, api
        self.dev = torch.device(device or "cuda:0")
        self.binn = binning
        self.k = int(k)
        self.qs = tuple(float(q) for q in qs)
        self.nq = len(self.qs)
        if not 1 <= self.nq <= api.MAX_LABEL_SETS:
            raise ValueError(f"1..{api.MAX_LABEL_SETS} q values per engine")
        self.tune = tune
        self.max_inflight = max_inflight
        # device bytes per voxel: int16 voxels + one uint8 label per q
        self.sched = Scheduler(2 + self.nq, hbm_budget, max_batch_voxels, max_batch_requests)
        self.s_h2d = torch.cuda.Stream(device=self.dev)
        self.s_cmp = torch.cuda.Stream(device=self.dev)
        self.s_d2h = torch.cuda.Stream(device=self.dev)
        self.inflight: Deque[dict] = collections.deque()
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, r: Request):
        self.sched.submit(r)

    def _launch(self, reqs: List[Request]) -> dict:
        torch, api = self.torch, self.api
        t_adm = self.now()
        dvols = []
        with torch.cuda.stream(self.s_h2d):
            for r in reqs:
                v = r.volume if isinstance(r.volume, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(r.volume))
                d = torch.empty(r.nvox, dtype=torch.int16, device=self.dev)
                d.copy_(v.reshape(-1), non_blocking=True)
                dvols.append(d)
        up = torch.cuda.Event()
        up.record(self.s_h2d)
        n = len(reqs)
        with torch.cuda.stream(self.s_cmp):
            self.s_cmp.wait_event(up)
            batch = api.Batch(dvols, device=self.dev, stream=self.s_cmp)
            hist = api.histogram(batch, self.binn, tune=self.tune, stream=self.s_cmp)
            P, Q = api.prefix(hist, self.qs, stream=self.s_cmp)
            thr, obj, st = api.threshold_search(P, Q, self.k, self.qs, tune=self.tune, stream=self.s_cmp)
            outs = api.label_sets(batch, self.binn, [thr[j] for j in range(self.nq)], self.k, tune=self.tune,
                                  stream=self.s_cmp)
        done_cmp = torch.cuda.Event()
        done_cmp.record(self.s_cmp)
        host = []
        with torch.cuda.stream(self.s_d2h):
            self.s_d2h.wait_event(done_cmp)
            for i in range(n):
                row = []
                for j in range(self.nq):
                    h = torch.empty(reqs[i].nvox, dtype=torch.uint8, pin_memory=True)
                    h.copy_(outs[j][i], non_blocking=True)
                    row.append(h)
                host.append(row)
            thr_h = torch.empty(thr.shape, dtype=thr.dtype, pin_memory=True)
            obj_h = torch.empty(obj.shape, dtype=obj.dtype, pin_memory=True)
            st_h = torch.empty(st.shape, dtype=st.dtype, pin_memory=True)
            thr_h.copy_(thr, non_blocking=True)
            obj_h.copy_(obj, non_blocking=True)
            st_h.copy_(st, non_blocking=True)
        fin = torch.cuda.Event()
        fin.record(self.s_d2h)
        # device tensors stay referenced until `fin` completes
        return dict(reqs=reqs, t_adm=t_adm, fin=fin, keep=(dvols, batch, hist, P, Q, thr, obj, st, outs),
                    host=host, thr=thr_h, obj=obj_h, st=st_h)

    def _retire(self, b: dict, results: List[Result]):
        t = self.now()
        thr = b["thr"].numpy()
        obj = b["obj"].numpy()
        st = b["st"].numpy()
        for i, r in enumerate(b["reqs"]):
            results.append(Result(r.rid, thr[:, i, :].copy(), obj[:, i].copy(), st[:, i].copy(), b["host"][i],
                                  r.arrival, b["t_adm"], t, r.nvox))
        self.sched.release(b["reqs"])

    def poll(self, results: List[Result], block: bool = False) -> int:
        """Retire finished batches (the oldest first); returns how many."""
        n = 0
        while self.inflight:
            b = self.inflight[0]
            if block:
                b["fin"].synchronize()
            elif not b["fin"].query():
                break
            self.inflight.popleft()
            self._retire(b, results)
            n += 1
            block = False
        return n

    def run(self, requests: Sequence[Request], realtime: bool = True) -> List[Result]:
        """Serve requests (arrival times on the engine clock, which starts
        now).  realtime=False makes every request arrive at once."""
        self.t0 = time.perf_counter()
        for r in sorted(requests, key=lambda r: r.arrival):
            if not realtime:
                r.arrival = 0.0
            self.submit(r)
        results: List[Result] = []
        while self.sched.queue or self.inflight:
            self.poll(results)
            if len(self.inflight) < self.max_inflight:
                reqs = self.sched.admit(self.now())
                if reqs:
                    self.inflight.append(self._launch(reqs))
                    continue
            nxt = self.sched.next_arrival()
            now = self.now()
            if self.inflight:
                if nxt is not None and nxt > now and len(self.inflight) < self.max_inflight:
                    time.sleep(min(1e-4, nxt - now))  # an arrival may come before the oldest batch ends
                else:
                    self.poll(results, block=True)  # frees a slot and its HBM budget
            elif nxt is None:
                break
            elif nxt > now:
                time.sleep(min(1e-3, nxt - now))
            else:  # cannot happen: submit() rejects requests over the budget
                raise RuntimeError(f"request {self.sched.queue[0].rid} cannot be admitted")
        return results
