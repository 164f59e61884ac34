"""Pins of the two-dimensional oracle (oracle/oracle2d.c) to facts other
than itself.  Every pin takes `lib` (an oracle-compatible library; None = the
oracle) so the mutation test can run them against planted mistakes:
a library correlation for the 3x3 mean, the one-dimensional oracle for the
marginals and for diagonal 2D histograms, closed forms for uniform 2D
histograms, symmetry and scaling invariances, the Shannon limit, and the
first-pair tie rule."""
import numpy as np
from scipy import ndimage

import oracle

QS = (0.3, 0.8, 1.5, 2.0)


def ln_q(x, q):
    return (x ** (1.0 - q) - 1.0) / (1.0 - q)


def _rand_h2(rng, L, zero_frac=0.5, hi=30):
    h = rng.integers(0, hi, (L, L)).astype(np.uint32)
    h[rng.random((L, L)) < zero_frac] = 0
    return h


def pin_mean3x3_library(lib=None):
    """The 3x3 floor mean equals a library correlation with edge repetition."""
    rng = np.random.default_rng(1)
    for H, W in [(1, 1), (1, 7), (5, 1), (3, 3), (17, 23), (64, 61)]:
        f = rng.integers(0, 4096, (H, W)).astype(np.int32)
        want = ndimage.correlate(f.astype(np.int64), np.ones((3, 3), np.int64), mode="nearest") // 9
        assert np.array_equal(oracle.mean3x3(f, lib=lib), want), (H, W)


def pin_mean3x3_constant_and_ramp(lib=None):
    f = np.full((6, 9), 41, np.int32)
    assert np.array_equal(oracle.mean3x3(f, lib=lib), f)
    ramp = np.tile(np.arange(9, dtype=np.int32) * 3, (6, 1))  # interior: mean of x-1, x, x+1 is x
    g = oracle.mean3x3(ramp, lib=lib)
    assert np.array_equal(g[:, 1:-1], ramp[:, 1:-1])
    assert g[0, 0] == (0 + 0 + 3) * 3 // 9  # edge repeated: columns 0, 0, 1


def pin_histogram2d_marginals(lib=None):
    rng = np.random.default_rng(2)
    img = rng.normal(-400, 500, (37, 45)).clip(-32768, 32767).astype(np.int16)
    lo, hi, L = -1024, -200, 64
    h2 = oracle.histogram2d(img, lo, hi, L, lib=lib)
    assert int(h2.sum()) == img.size
    # rows: the one-dimensional histogram (an independent routine)
    assert np.array_equal(h2.sum(axis=1), oracle.histogram(img.reshape(-1), lo, hi, L, lib=lib))
    # columns: the 3x3 floor mean of the gray levels from a library correlation
    f = np.array([oracle.bin_of(v, lo, hi, L) for v in img.reshape(-1)], np.int64).reshape(img.shape)
    g = ndimage.correlate(f, np.ones((3, 3), np.int64), mode="nearest") // 9
    assert np.array_equal(h2.sum(axis=0), np.bincount(g.reshape(-1), minlength=L))


def pin_direct_and_prefix_modes_agree(lib=None):
    for q in QS:
        rng = np.random.default_rng(int(q * 100))
        for L in (2, 3, 7, 16):
            h = _rand_h2(rng, L)
            for t in range(L - 1):
                for s in range(L - 1):
                    a = oracle.objective2d(h, t, s, q, oracle.MODE_DIRECT, lib=lib)
                    b = oracle.objective2d(h, t, s, q, oracle.MODE_PREFIX, lib=lib)
                    assert (np.isnan(a) and np.isnan(b)) or abs(a - b) <= 1e-12 * max(1.0, abs(a)), (q, L, t, s)
            ra = oracle.search2d(h, q, oracle.MODE_DIRECT, lib=lib)
            rb = oracle.search2d(h, q, oracle.MODE_PREFIX, lib=lib)
            assert ra.status == rb.status
            if ra.status == oracle.OK and ra.rel_gap() > 1e-9:
                assert ra.thr.tolist() == rb.thr.tolist()


def pin_diagonal_reduces_to_1d(lib=None):
    """With all mass on the diagonal (g == f) the classes of (t, t) are the
    one-dimensional classes of threshold t."""
    for q in QS:
        rng = np.random.default_rng(7 + int(q * 10))
        L = 24
        c = rng.integers(0, 50, L).astype(np.uint32)
        c[rng.random(L) < 0.3] = 0
        h2 = np.diag(c).astype(np.uint32)
        for mode in (oracle.MODE_DIRECT, oracle.MODE_PREFIX):
            for t in range(L - 1):
                a = oracle.objective2d(h2, t, t, q, mode, lib=lib)
                b = oracle.objective(c, np.array([t], np.int32), q, oracle.MODE_DIRECT, lib=lib)
                assert (np.isnan(a) and not np.isfinite(b)) or abs(a - b) <= 1e-12 * max(1.0, abs(b)), (q, t)


def pin_uniform_closed_form(lib=None):
    """Uniform 2D histogram: class entropies ln_q(m) for m cells, composed by
    the pseudo-additive rule into ln_q(m1 m2); (t+1)(s+1)(L-1-t)(L-1-s) is
    largest at t = s = L/2 - 1 for even L."""
    L = 10
    h2 = np.full((L, L), 5, np.uint32)
    for q in QS:
        for mode in (oracle.MODE_DIRECT, oracle.MODE_PREFIX):
            for t in range(L - 1):
                for s in range(L - 1):
                    m1, m2 = (t + 1) * (s + 1), (L - 1 - t) * (L - 1 - s)
                    want = ln_q(float(m1 * m2), q)
                    got = oracle.objective2d(h2, t, s, q, mode, lib=lib)
                    assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (q, t, s, got, want)
            r = oracle.search2d(h2, q, mode, lib=lib)
            assert r.status == oracle.OK and r.thr.tolist() == [L // 2 - 1, L // 2 - 1]


def pin_transpose_and_scaling(lib=None):
    for q in QS:
        rng = np.random.default_rng(99 + int(q * 10))
        L = 12
        h = _rand_h2(rng, L, zero_frac=0.3)
        ht = np.ascontiguousarray(h.T)
        for t in range(L - 1):
            for s in range(L - 1):
                a = oracle.objective2d(h, t, s, q, lib=lib)
                b = oracle.objective2d(ht, s, t, q, lib=lib)
                assert (np.isnan(a) and np.isnan(b)) or abs(a - b) <= 1e-12 * max(1.0, abs(a))
        r, r3 = oracle.search2d(h, q, lib=lib), oracle.search2d(h * 3, q, lib=lib)
        assert r.thr.tolist() == r3.thr.tolist() and abs(r.obj - r3.obj) <= 1e-12 * abs(r.obj)
        rt = oracle.search2d(ht, q, lib=lib)
        if r.rel_gap() > 1e-9:
            assert rt.thr.tolist() == r.thr.tolist()[::-1]


def pin_shannon_limit(lib=None):
    rng = np.random.default_rng(5)
    h = _rand_h2(rng, 14, zero_frac=0.3)
    k = oracle.search2d(h, 1.0, oracle.MODE_KAPUR, lib=lib)
    for q in (1.0 - 1e-6, 1.0 + 1e-6):
        r = oracle.search2d(h, q, oracle.MODE_PREFIX, lib=lib)
        assert abs(r.obj - k.obj) <= 1e-4 * abs(k.obj)
        if k.rel_gap() > 1e-4:
            assert r.thr.tolist() == k.thr.tolist()


def pin_degenerate_empty_and_first_pair(lib=None):
    L = 8
    h = np.zeros((L, L), np.uint32)
    assert oracle.search2d(h, 0.8, lib=lib).status == oracle.EMPTY
    h[3, 4] = 10  # one cell: one of the two classes is always empty
    assert oracle.search2d(h, 0.8, lib=lib).status == oracle.DEGENERATE
    h[6, 6] = 4  # valid pairs: t in 3..5, s in 4..5, all with two one-cell classes (S = 0)
    for mode in (oracle.MODE_DIRECT, oracle.MODE_PREFIX):
        r = oracle.search2d(h, 0.8, mode, lib=lib)
        assert r.status == oracle.OK and r.obj == 0.0
        assert r.thr.tolist() == [3, 4]  # the first of the tied pairs


ALL_PINS = [pin_mean3x3_library, pin_mean3x3_constant_and_ramp, pin_histogram2d_marginals,
            pin_direct_and_prefix_modes_agree, pin_diagonal_reduces_to_1d, pin_uniform_closed_form,
            pin_transpose_and_scaling, pin_shannon_limit, pin_degenerate_empty_and_first_pair]
