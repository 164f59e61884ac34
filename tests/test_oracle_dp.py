"""The oracle's dynamic-programming search (oracle.search_dp), which reaches
numbers of thresholds the exhaustive oracle cannot (k = 4 over 1024 levels),
pinned against the exhaustive oracle on every tuple of small histograms, the
uniform closed form with its first-tuple tie rule, and the degenerate and
empty cases."""
import math

import numpy as np
import pytest

import oracle


def _close(a, b, rel=1e-12):
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-300)


@pytest.mark.parametrize("q", [0.3, 0.8, 1.5, 3.0, 1.0])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_dp_equals_exhaustive_on_small_histograms(k, q):
    mode = oracle.MODE_KAPUR if q == 1.0 else oracle.MODE_PREFIX
    rng = np.random.default_rng(100 * k + int(10 * q))
    for trial in range(12):
        L = int(rng.integers(k + 1, 25))
        h = rng.integers(0, 60, L).astype(np.uint32)
        h[rng.random(L) < 0.25] = 0  # runs of empty bins: exact ties
        ex = oracle.search(h, k, q, mode)
        dp = oracle.search_dp(h, k, q, mode)
        assert dp.status == ex.status, (h, k, q, ex, dp)
        if ex.status != oracle.OK:
            assert dp.thr.tolist() == [-1] * k
            continue
        assert _close(dp.obj, ex.obj), (h, k, q, ex, dp)
        if dp.thr.tolist() != ex.thr.tolist():
            # only a tie up to FP64 rounding may pick another tuple
            s = oracle.objective(h, dp.thr, q, mode)
            assert _close(s, ex.obj), (h, k, q, ex, dp, s)


def test_dp_k4_on_48_levels():
    rng = np.random.default_rng(7)
    h = rng.integers(0, 1000, 48).astype(np.uint32)
    for q in (0.5, 2.0):
        ex = oracle.search(h, 4, q)
        dp = oracle.search_dp(h, 4, q)
        assert dp.thr.tolist() == ex.thr.tolist() and _close(dp.obj, ex.obj), (q, ex, dp)


def test_dp_uniform_closed_form():
    """20 equal bins, four thresholds: the product of the class sizes (bins)
    is largest for five classes of 4, S = ln_q(4^5), and the first such tuple
    is (3, 7, 11, 15)."""
    h = np.full(20, 5, dtype=np.uint32)
    q = 0.8
    dp = oracle.search_dp(h, 4, q)
    want = (1024.0 ** (1.0 - q) - 1.0) / (1.0 - q)
    assert dp.thr.tolist() == [3, 7, 11, 15], dp
    assert math.isclose(dp.obj, want, rel_tol=1e-12), (dp.obj, want)


def test_dp_degenerate_and_empty():
    h = np.zeros(30, dtype=np.uint32)
    assert oracle.search_dp(h, 2, 0.8).status == oracle.EMPTY
    h[[4, 9, 20]] = 7  # three occupied bins: no valid tuple of four classes
    r = oracle.search_dp(h, 3, 0.8)
    assert r.status == oracle.DEGENERATE and r.thr.tolist() == [-1, -1, -1]
    r2 = oracle.search_dp(h, 2, 0.8)  # exactly k + 1 occupied bins: S* = 0, the first tuple
    ex = oracle.search(h, 2, 0.8)
    assert r2.status == oracle.OK and r2.thr.tolist() == ex.thr.tolist() and abs(r2.obj) < 1e-12
