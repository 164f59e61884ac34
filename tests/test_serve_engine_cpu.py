"""The serving loop on the CPU with an oracle-backed fake backend (no GPU):
every request answered once and equal to its result alone, batches within
the caps, admission by the device bytes the backend reports free, a request
that can never fit refused instead of deadlocking, and failures isolated: a
request whose launch or collection fails gets an error, the others of its
batch are served and the loop goes on.  Also the pinned-buffer pool."""
import time

import numpy as np
import pytest

import oracle
from paper_2012_10684_amd import synth
from paper_2012_10684_amd.serve import Engine, PinnedPool, Request

LO, HI, L, K, QS = -1024, 3071, 512, 2, (0.8, 1.5)


class OracleBackend:
    """Same interface as GpuBackend; computes with the oracle at launch, and
    makes a batch ready `delay` seconds later.  Device memory is simulated:
    a launched batch holds 4 bytes per voxel until it is collected."""

    def __init__(self, free=1 << 40, fail_launch=(), fail_collect=(), delay=0.0):
        self.free = free
        self.held = 0
        self.fail_launch, self.fail_collect = set(fail_launch), set(fail_collect)
        self.delay = delay
        self.batches = []

    def free_bytes(self):
        return self.free - self.held

    def launch(self, reqs):
        bad = [r.rid for r in reqs if r.rid in self.fail_launch]
        if bad:
            raise RuntimeError(f"injected launch failure for {bad}")
        self.batches.append([r.rid for r in reqs])
        out = []
        for r in reqs:
            v = np.asarray(r.volume)
            h = oracle.histogram(v, LO, HI, L)
            res = [oracle.search(h, K, q) for q in QS]
            out.append(dict(thr=np.stack([x.thr for x in res]), obj=np.array([x.obj for x in res]),
                            status=np.array([x.status for x in res], np.int32),
                            labels=[oracle.label(v.reshape(-1), LO, HI, L, x.thr) for x in res],
                            device_s=0.001, kernels_s=0.0005))
        held = 4 * sum(r.nvox for r in reqs)
        self.held += held
        return dict(t=time.perf_counter(), out=out, held=held, rids=[r.rid for r in reqs])

    def ready(self, h):
        return time.perf_counter() >= h["t"] + self.delay

    def wait(self, h):
        while not self.ready(h):
            time.sleep(1e-4)

    def collect(self, h):
        self.held -= h["held"]
        if set(h["rids"]) & self.fail_collect:
            raise RuntimeError("injected failure while collecting")
        return h["out"]

    def release(self, res):
        res.labels = []


@pytest.fixture(scope="module")
def vols():
    return [synth.make_volume(synth.rng_for(5, 950 + i), 2 + i % 3, 64) for i in range(7)]


def _alone(v):
    h = oracle.histogram(v, LO, HI, L)
    return [oracle.search(h, K, q).thr.tolist() for q in QS]


def test_every_request_once_and_equal_to_alone(vols):
    be = OracleBackend(delay=0.002)
    eng = Engine(k=K, qs=QS, backend=be, max_batch_requests=3, max_inflight=2)
    seen = []
    res = eng.run([Request(i, v, 0.001 * i) for i, v in enumerate(vols)], realtime=True, on_result=seen.append)
    assert sorted(r.rid for r in res) == list(range(len(vols)))
    assert [r.rid for r in seen] == [r.rid for r in res]  # the callback saw each result once, in order
    assert all(len(b) <= 3 for b in be.batches)
    for r in res:
        assert r.error is None and r.thr.tolist() == _alone(vols[r.rid])
        assert r.done >= r.admitted >= r.arrival - 1e-9 and r.device_s == 0.001


def test_admission_follows_free_device_bytes(vols):
    per = 4 * 2 * 64 * 64  # the fake backend holds 4 B/voxel; the engine's cost is (2 + nq) B/voxel
    be = OracleBackend(free=2 * per + 10, delay=0.003)
    eng = Engine(k=K, qs=QS, backend=be, max_batch_requests=64, max_inflight=2)
    small = [synth.make_volume(synth.rng_for(5, 990 + i), 2, 64) for i in range(6)]
    res = eng.run([Request(i, v, 0.0) for i, v in enumerate(small)], realtime=False)
    assert sorted(r.rid for r in res) == list(range(6)) and all(r.error is None for r in res)
    # cost 4 x 8192 = 32 KiB of the 64 KiB free at first: two per batch, then what the held memory leaves
    assert max(len(b) for b in be.batches) <= 2 and len(be.batches) >= 3


def test_request_that_can_never_fit_is_refused(vols):
    be = OracleBackend(free=4 * 64 * 64 * 3)  # room for 3 slices of 64 x 64 at 4 B/voxel
    eng = Engine(k=K, qs=QS, backend=be)
    big = synth.make_volume(synth.rng_for(5, 980), 5, 64)  # 5 slices: never fits
    res = {r.rid: r for r in eng.run([Request(0, vols[0], 0.0), Request(1, big, 0.0), Request(2, vols[3], 0.0)],
                                     realtime=False)}
    assert res[1].error and "free" in res[1].error
    assert res[0].error is None and res[2].error is None
    assert eng.refused == 1


def test_failing_launch_fails_alone(vols):
    be = OracleBackend(fail_launch={3})
    eng = Engine(k=K, qs=QS, backend=be, max_batch_requests=64)
    res = {r.rid: r for r in eng.run([Request(i, v, 0.0) for i, v in enumerate(vols)], realtime=False)}
    assert sorted(res) == list(range(len(vols)))
    assert "injected launch failure" in res[3].error and res[3].thr is None
    for i in set(range(len(vols))) - {3}:
        assert res[i].error is None and res[i].thr.tolist() == _alone(vols[i])
    assert eng.sched.inflight_bytes == 0


def test_failing_collection_fails_its_batch_only(vols):
    be = OracleBackend(fail_collect={1}, delay=0.001)
    eng = Engine(k=K, qs=QS, backend=be, max_batch_requests=2, max_inflight=1)
    res = {r.rid: r for r in eng.run([Request(i, v, 0.0) for i, v in enumerate(vols[:5])], realtime=False)}
    batch_of_1 = next(b for b in be.batches if 1 in b)
    for i in range(5):
        if i in batch_of_1:
            assert res[i].error and "collecting" in res[i].error
        else:
            assert res[i].error is None and res[i].thr.tolist() == _alone(vols[i])


def test_bad_requests_are_answered_with_errors(vols):
    eng = Engine(k=K, qs=QS, backend=OracleBackend(), hbm_budget=4 * 64 * 64 * 4)
    f32 = vols[0].astype(np.float32)
    too_big = synth.make_volume(synth.rng_for(5, 981), 5, 64)  # 5 x 4096 voxels x 4 B > the fixed budget
    res = {r.rid: r for r in eng.run([Request(0, f32, 0.0), Request(1, vols[1], 0.0), Request(2, too_big, 0.0)],
                                     realtime=False)}
    assert "int16" in res[0].error
    assert "budget" in res[2].error
    assert res[1].error is None


def test_pinned_pool_reuses_and_overflows():
    made = []

    def alloc(n):
        made.append(n)
        return np.zeros(n, np.uint8)

    p = PinnedPool(2, 100, alloc)
    a, b = p.take(10), p.take(100)
    assert len(made) == 2 and a.size == 10 and b.size == 100
    c = p.take(5)  # pool empty: a fresh buffer
    assert p.extra == 1 and len(made) == 3
    p.give(a)
    d = p.take(50)
    assert p.extra == 1 and d.size == 50 and len(made) == 3  # a's slot again
    big = p.take(500)  # larger than a slot
    assert big.size == 500 and p.extra == 2
    p.give(c)  # not from the pool: ignored
    assert len(p.free) == 0
