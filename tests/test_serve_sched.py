"""Serving scheduler on the CPU: FIFO admission, voxel / request / HBM
budgets, release, ordering errors and latency statistics (no GPU)."""
import numpy as np
import pytest

from paper_2012_10684_amd.serve import Request, Result, Scheduler, latency_stats


class Vol:
    """Stand-in for a volume: only the shape is read by the scheduler."""

    def __init__(self, n):
        self.shape = (n,)


def req(i, n, t):
    return Request(i, Vol(n), t)


def test_fifo_and_arrival_gate():
    s = Scheduler(5, hbm_budget=10_000, max_batch_voxels=1_000)
    for i, (n, t) in enumerate([(100, 0.0), (200, 0.1), (300, 0.5)]):
        s.submit(req(i, n, t))
    assert [r.rid for r in s.admit(0.05)] == [0]
    assert [r.rid for r in s.admit(0.2)] == [1]
    assert s.admit(0.3) == []
    assert s.next_arrival() == 0.5
    assert [r.rid for r in s.admit(1.0)] == [2]
    assert s.next_arrival() is None


def test_voxel_and_request_caps():
    s = Scheduler(1, hbm_budget=1 << 40, max_batch_voxels=500, max_batch_requests=3)
    for i in range(6):
        s.submit(req(i, 200, 0.0))
    assert [r.rid for r in s.admit(0)] == [0, 1]  # a third would exceed 500 voxels
    s2 = Scheduler(1, hbm_budget=1 << 40, max_batch_voxels=10_000, max_batch_requests=3)
    for i in range(6):
        s2.submit(req(i, 200, 0.0))
    assert [r.rid for r in s2.admit(0)] == [0, 1, 2]
    assert [r.rid for r in s2.admit(0)] == [3, 4, 5]


def test_oversized_request_is_admitted_alone():
    s = Scheduler(1, hbm_budget=1 << 40, max_batch_voxels=100)
    s.submit(req(0, 1000, 0.0))
    s.submit(req(1, 10, 0.0))
    assert [r.rid for r in s.admit(0)] == [0]
    assert [r.rid for r in s.admit(0)] == [1]


def test_hbm_budget_and_release():
    s = Scheduler(3, hbm_budget=3000, max_batch_voxels=10_000)
    for i in range(4):
        s.submit(req(i, 400, 0.0))  # 1200 bytes each
    a = s.admit(0)
    assert [r.rid for r in a] == [0, 1]
    assert s.inflight_bytes == 2400
    assert s.admit(0) == []  # head needs 1200, only 600 left
    s.release(a[:1])
    assert [r.rid for r in s.admit(0)] == [2]
    s.release(a[1:])
    assert [r.rid for r in s.admit(0)] == [3]


def test_errors():
    s = Scheduler(2, hbm_budget=100, max_batch_voxels=10)
    with pytest.raises(ValueError):
        s.submit(req(0, 51, 0.0))  # 102 bytes > budget
    s.submit(req(1, 5, 1.0))
    with pytest.raises(ValueError):
        s.submit(req(2, 5, 0.5))  # out of arrival order
    with pytest.raises(ValueError):
        Scheduler(0, 1, 1)


def test_latency_stats():
    rs = [Result(i, None, None, None, [], arrival=0.0, admitted=0.0, done=0.01 * (i + 1), nvox=100)
          for i in range(100)]
    st = latency_stats(rs, wall=2.0)
    assert st["n"] == 100
    assert st["p50_s"] == pytest.approx(np.percentile(np.arange(1, 101) * 0.01, 50))
    assert st["p99_s"] == pytest.approx(np.percentile(np.arange(1, 101) * 0.01, 99))
    assert st["max_s"] == pytest.approx(1.0)
    assert st["voxels_per_s"] == pytest.approx(100 * 100 / 2.0)
    assert latency_stats([]) == {"n": 0, "errors": 0}
    # failed requests are counted, not timed
    bad = Result(7, None, None, None, [], arrival=0.0, admitted=0.0, done=9.0, nvox=100, error="refused")
    st2 = latency_stats(rs + [bad], wall=2.0)
    assert st2["n"] == 100 and st2["errors"] == 1 and st2["max_s"] == pytest.approx(1.0)


def test_admission_by_free_device_bytes():
    """Without a fixed budget the requests admitted together must fit in the
    device bytes free at that moment."""
    s = Scheduler(3, None, max_batch_voxels=10_000)
    for i in range(4):
        s.submit(req(i, 400, 0.0))  # 1200 bytes each
    assert [r.rid for r in s.admit(0, free_bytes=2500)] == [0, 1]
    assert s.admit(0, free_bytes=1000) == []
    assert [r.rid for r in s.admit(0, free_bytes=1200)] == [2]
    assert [r.rid for r in s.admit(0)] == [3]  # no figure: only the other budgets
