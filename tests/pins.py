"""Pins for the CPU oracle: checks against facts the paper and mathematics fix,
independent of the oracle's own formulas.

Each ``pin_*`` takes ``lib`` (None = the real oracle, or a mutated copy loaded
by the mutation tests) and raises AssertionError on a violation.  They are
kept small so that every pin runs in well under a second.

What pins what:
  bin map        -- closed form b(v) = v + 1024 on the 4096-bin [-1024, 3071]
                    window; an integer edge search (v in bin i iff
                    i*W <= (v-lo)*L < (i+1)*W) over every int16 value.
  histogram      -- np.bincount of the edge-search bins; sum of counts = n.
  objective      -- uniform histograms: S = ln_q(prod m_j) (closed form,
                    derived in tests/golden/uniform_closed_form.txt); q = 2:
                    Gini-Simpson product S = 1 - prod_j sum (p/w)^2;
                    q -> 1: Kapur's sum of class Shannon entropies computed by
                    scipy.stats.entropy; a dynamic programme (a different
                    algorithm over the product identity) reaches the same
                    maximum.
  arg max        -- closed-form optimum on uniform histograms and on
                    histograms with exactly k+1 occupied bins (ties broken to
                    the first tuple); mirror symmetry; invariance under
                    scaling the counts and under padding with empty bins.
  labels         -- np.searchsorted(thr, b, side='left').
"""
from __future__ import annotations

import itertools
from decimal import Decimal, getcontext

import numpy as np
import scipy.stats

import oracle

getcontext().prec = 50

HU_LO, HU_HI = -32768, 32767


def ln_q(x: float, q: float) -> float:
    """q-logarithm (x^(1-q) - 1)/(1-q), evaluated with 50-digit decimals."""
    X = Decimal(x)
    e = Decimal(1) - Decimal(repr(q))
    return float((X ** e - Decimal(1)) / e)


def edge_bins(v: np.ndarray, lo: int, hi: int, L: int) -> np.ndarray:
    """Bin of each value found by searching integer edges: in-window v lies in
    bin i iff i*W <= (v-lo)*L < (i+1)*W; below the window -> 0, above -> L-1."""
    W = hi - lo + 1
    v = np.asarray(v, dtype=np.int64)
    x = (np.clip(v, lo, hi) - lo) * L
    edges = np.arange(L + 1, dtype=np.int64) * W
    b = np.searchsorted(edges, x, side="right") - 1
    b = np.where(v < lo, 0, b)
    b = np.where(v > hi, L - 1, b)
    return b


def all_int16() -> np.ndarray:
    return np.arange(HU_LO, HU_HI + 1, dtype=np.int64).astype(np.int16)


# ---------------------------------------------------------------- bin map

def pin_binmap_identity(lib=None):
    v = all_int16()
    b = oracle.bin_map(v, -1024, 3071, 4096, lib=lib)
    want = np.clip(v.astype(np.int64), -1024, 3071) + 1024
    assert np.array_equal(b, want), "4096-bin window [-1024,3071] must map v -> v+1024"


WINDOWS = [(-1024, 3071, 1024), (-1024, -200, 256), (-1024, 3071, 512), (-1024, -1000, 256),
           (-5, 7, 13), (100, 100, 4), (-32768, 32767, 4096), (3, 1000, 7)]


def pin_binmap_edges(lib=None):
    v = all_int16()
    for lo, hi, L in WINDOWS:
        b = oracle.bin_map(v, lo, hi, L, lib=lib)
        assert np.array_equal(b, edge_bins(v, lo, hi, L)), f"bin map differs from edge search for {(lo, hi, L)}"


def pin_histogram(lib=None):
    rng = np.random.default_rng(7)
    for lo, hi, L in WINDOWS:
        n = int(rng.integers(0, 5000))
        v = rng.integers(-2000, 4000, n).astype(np.int16)
        h = oracle.histogram(v, lo, hi, L, lib=lib)
        assert int(h.sum()) == n, "histogram counts must sum to the voxel count"
        want = np.bincount(edge_bins(v, lo, hi, L), minlength=L)
        assert np.array_equal(h, want.astype(np.uint32)), f"histogram differs from bincount for {(lo, hi, L)}"


# ---------------------------------------------------------------- objective

def _tuples(L, k):
    return itertools.combinations(range(L - 1), k)


def _class_sizes(L, t):
    edges = [-1] + list(t) + [L - 1]
    return [edges[j + 1] - edges[j] for j in range(len(t) + 1)]


def pin_uniform_closed_form(lib=None, mode=oracle.MODE_PREFIX):
    rng = np.random.default_rng(11)
    for L, k, q in [(4, 1, 0.8), (10, 2, 0.5), (9, 3, 1.5), (12, 2, 2.0), (7, 1, 0.3), (16, 3, 0.8)]:
        h = np.full(L, int(rng.integers(1, 9)), dtype=np.uint32)
        for t in _tuples(L, k):
            m = int(np.prod(_class_sizes(L, t)))
            S = oracle.objective(h, t, q, mode, lib=lib)
            want = ln_q(m, q)
            assert abs(S - want) <= 1e-12 * max(1.0, abs(want)), f"uniform L={L} k={k} q={q} t={t}: {S} vs {want}"


def pin_uniform_argmax(lib=None, mode=oracle.MODE_PREFIX):
    # L=4, k=1: sizes (2,2) beat (1,3), (3,1); S* = ln_q(4).
    r = oracle.search(np.ones(4, np.uint32), 1, 0.8, mode, lib=lib)
    assert r.status == oracle.OK and r.thr.tolist() == [1], r
    assert abs(r.obj - ln_q(4, 0.8)) <= 1e-13, r
    assert abs(r.second - ln_q(3, 0.8)) <= 1e-13, r
    # L=10, k=2: the optimum is any tuple with class sizes {3,3,4}, S* = ln_q(36).
    for q in (0.5, 0.8, 1.5):
        r = oracle.search(np.ones(10, np.uint32), 2, q, mode, lib=lib)
        assert sorted(_class_sizes(10, r.thr.tolist())) == [3, 3, 4], r
        assert abs(r.obj - ln_q(36, q)) <= 1e-12 * max(1, abs(r.obj)), r
    # q < 1 and q > 1 both pick the balanced split on a uniform histogram
    r = oracle.search(np.ones(6, np.uint32), 1, 1.7, mode, lib=lib)
    assert r.thr.tolist() == [2], r


def pin_separated_bins(lib=None, mode=oracle.MODE_PREFIX):
    """Exactly k+1 occupied bins: every valid tuple puts one occupied bin in
    each class, so S = 0 for all of them and the first tuple in lexicographic
    order wins: t_j = position of the j-th occupied bin."""
    rng = np.random.default_rng(3)
    cases = [(16, 1, [3, 9]), (16, 2, [0, 5, 15]), (20, 3, [2, 3, 11, 19]), (8, 1, [6, 7]), (8, 2, [0, 1, 2])]
    for L, k, occ in cases:
        h = np.zeros(L, np.uint32)
        h[occ] = rng.integers(1, 100, len(occ))
        for q in (0.5, 1.5):
            r = oracle.search(h, k, q, mode, lib=lib)
            assert r.status == oracle.OK, (L, k, occ, r)
            assert r.thr.tolist() == occ[:k], (L, k, occ, q, r)
            assert abs(r.obj) <= 1e-12, (L, k, occ, q, r)
    # fewer than k+1 occupied bins: no valid tuple
    h = np.zeros(12, np.uint32)
    h[[4, 8]] = 5
    r = oracle.search(h, 2, 0.8, mode, lib=lib)
    assert r.status == oracle.DEGENERATE and r.thr.tolist() == [-1, -1], r
    r = oracle.search(np.zeros(12, np.uint32), 1, 0.8, mode, lib=lib)
    assert r.status == oracle.EMPTY, r


def _gini_simpson(h, t):
    p = h / h.sum()
    edges = [-1] + list(t) + [len(h) - 1]
    prod = 1.0
    for j in range(len(t) + 1):
        c = p[edges[j] + 1: edges[j + 1] + 1]
        w = c.sum()
        prod *= float(np.sum((c / w) ** 2))
    return 1.0 - prod


def pin_q2_gini_simpson(lib=None, mode=oracle.MODE_PREFIX):
    rng = np.random.default_rng(5)
    for L, k in [(8, 1), (10, 2), (9, 3)]:
        h = rng.integers(1, 50, L).astype(np.uint32)
        for t in _tuples(L, k):
            S = oracle.objective(h, t, 2.0, mode, lib=lib)
            assert abs(S - _gini_simpson(h, t)) <= 1e-12, (L, k, t)


def _kapur(h, t):
    edges = [-1] + list(t) + [len(h) - 1]
    return sum(float(scipy.stats.entropy(h[edges[j] + 1: edges[j + 1] + 1].astype(np.float64)))
               for j in range(len(t) + 1))


def pin_kapur_limit(lib=None, mode=oracle.MODE_PREFIX):
    rng = np.random.default_rng(9)
    for L, k in [(12, 1), (10, 2), (9, 3)]:
        h = rng.integers(1, 200, L).astype(np.uint32)
        for t in _tuples(L, k):
            K = _kapur(h, t)
            assert abs(oracle.objective(h, t, 1.0, oracle.MODE_KAPUR, lib=lib) - K) <= 1e-12, (L, k, t)
            for q in (1.0 - 1e-6, 1.0 + 1e-6):
                S = oracle.objective(h, t, q, mode, lib=lib)
                assert abs(S - K) <= 1e-5 * (1.0 + K) ** 2, (L, k, t, q, S, K)
    # the arg max agrees with Kapur's when Kapur's optimum is well separated
    h = rng.integers(1, 200, 24).astype(np.uint32)
    h[10:14] += 400
    kr = oracle.search(h, 1, 1.0, oracle.MODE_KAPUR, lib=lib)
    assert kr.rel_gap() > 1e-4
    for q in (1.0 - 1e-6, 1.0 + 1e-6):
        r = oracle.search(h, 1, q, mode, lib=lib)
        assert r.thr.tolist() == kr.thr.tolist(), (q, r, kr)


def _dp_max(h, k, q):
    """max over tuples of Lambda = sum_j [ln sum c^q - q ln sum c] (natural
    logs; N cancels), by dynamic programming over the last class boundary."""
    L = len(h)
    c = h.astype(np.float64)
    s = 1.0 if q < 1 else -1.0
    term = np.full((L, L), -np.inf)
    for a in range(L):
        for b in range(a, L):
            m = c[a:b + 1]
            if m.sum() > 0:
                term[a, b] = s * (np.log(np.sum(m[m > 0] ** q)) - q * np.log(m.sum()))
    best = term[0].copy()  # one class ending at b
    for _ in range(k):
        nxt = np.full(L, -np.inf)
        for b in range(L):
            nxt[b] = np.max(best[:b] + term[1:b + 1, b]) if b > 0 else -np.inf
        best = nxt
    lam = s * best[L - 1]
    return np.expm1(lam) / (1.0 - q)


def pin_dp(lib=None, mode=oracle.MODE_PREFIX):
    rng = np.random.default_rng(13)
    for L, k, q in [(12, 1, 0.8), (14, 2, 0.5), (13, 3, 1.5), (16, 2, 2.5), (11, 3, 0.3)]:
        h = rng.integers(0, 40, L).astype(np.uint32)
        h[rng.integers(0, L, 2)] = 0
        r = oracle.search(h, k, q, mode, lib=lib)
        want = _dp_max(h, k, q)
        assert abs(r.obj - want) <= 1e-11 * max(1.0, abs(want)), (L, k, q, r, want)


def pin_search_dp(lib=None):
    """The oracle's dynamic-programming search: the same maximum as the
    independent numpy dynamic programme over the log form (k up to 5, 40
    levels, beyond the exhaustive search's reach at these sizes), the same
    tuple and value as the exhaustive search on small histograms, and the
    uniform closed form with its first-tuple tie rule (20 equal bins, four
    thresholds: classes of 4 bins, S = ln_q(4^5), tuple (3, 7, 11, 15))."""
    rng = np.random.default_rng(17)
    for L, k, q in [(40, 4, 0.8), (36, 5, 1.5), (30, 4, 0.5)]:
        h = rng.integers(0, 500, L).astype(np.uint32)
        h[rng.integers(0, L, 3)] = 0
        r = oracle.search_dp(h, k, q, lib=lib)
        want = _dp_max(h, k, q)
        assert r.status == oracle.OK and abs(r.obj - want) <= 1e-11 * max(1.0, abs(want)), (L, k, q, r, want)
        assert abs(oracle.objective(h, r.thr, q, lib=lib) - r.obj) <= 1e-11 * max(1.0, abs(r.obj)), (L, k, q, r)
    for L, k, q in [(14, 2, 0.8), (16, 3, 1.5), (18, 4, 0.5)]:
        h = rng.integers(0, 40, L).astype(np.uint32)
        h[rng.integers(0, L, 2)] = 0
        ex = oracle.search(h, k, q, lib=lib)
        r = oracle.search_dp(h, k, q, lib=lib)
        assert r.thr.tolist() == ex.thr.tolist() or ex.rel_gap() < 1e-9, (L, k, q, ex, r)
        assert abs(r.obj - ex.obj) <= 1e-12 * max(1.0, abs(ex.obj)), (L, k, q, ex, r)
    u = oracle.search_dp(np.full(20, 5, dtype=np.uint32), 4, 0.8, lib=lib)
    assert u.thr.tolist() == [3, 7, 11, 15], u
    assert abs(u.obj - ln_q(4.0 ** 5, 0.8)) <= 1e-12 * abs(u.obj), u
    # runs of empty bins: thresholds anywhere in a run tie exactly; the first
    # tuple wins, as in the exhaustive search
    h = np.array([7, 3, 0, 0, 0, 9, 2, 0, 0, 4, 6, 0, 0, 5], dtype=np.uint32)
    for k in (1, 2, 3):
        ex = oracle.search(h, k, 0.8, lib=lib)
        r = oracle.search_dp(h, k, 0.8, lib=lib)
        assert r.thr.tolist() == ex.thr.tolist(), (k, ex, r)
    # the last k + 1 bins occupied, one per class: the only valid tuple is
    # (L-k-1, ..., L-2), every class boundary at its upper limit
    L, k = 15, 4
    h = np.zeros(L, dtype=np.uint32)
    h[L - k - 1:] = 5
    r = oracle.search_dp(h, k, 0.8, lib=lib)
    assert r.status == oracle.OK and r.thr.tolist() == list(range(L - k - 1, L - 1)), r


def pin_symmetry(lib=None, mode=oracle.MODE_PREFIX):
    rng = np.random.default_rng(17)
    for L, k, q in [(16, 1, 0.8), (14, 2, 0.5), (12, 3, 1.5)]:
        half = rng.integers(0, 30, L // 2).astype(np.uint32)
        h = np.concatenate([half, half[::-1]])
        for t in _tuples(L, k):
            mt = tuple(sorted(L - 2 - x for x in t))
            a = oracle.objective(h, t, q, mode, lib=lib)
            b = oracle.objective(h, mt, q, mode, lib=lib)
            assert (np.isnan(a) and np.isnan(b)) or abs(a - b) <= 1e-12 * max(1, abs(a)), (t, mt, a, b)
        r = oracle.search(h, k, q, mode, lib=lib)
        mt = sorted(L - 2 - x for x in r.thr.tolist())
        assert abs(oracle.objective(h, mt, q, mode, lib=lib) - r.obj) <= 1e-12 * max(1, abs(r.obj))


def pin_invariances(lib=None, mode=oracle.MODE_PREFIX):
    rng = np.random.default_rng(19)
    for L, k, q in [(20, 1, 0.8), (15, 2, 1.5), (12, 3, 0.5)]:
        h = rng.integers(0, 60, L).astype(np.uint32)
        r = oracle.search(h, k, q, mode, lib=lib)
        r3 = oracle.search(h * 3, k, q, mode, lib=lib)
        assert r3.thr.tolist() == r.thr.tolist() and abs(r3.obj - r.obj) <= 1e-12 * max(1, abs(r.obj))
        e = 3
        hp = np.concatenate([np.zeros(e, np.uint32), h])
        rp = oracle.search(hp, k, q, mode, lib=lib)
        assert rp.thr.tolist() == [x + e for x in r.thr.tolist()], (r, rp)
        assert abs(rp.obj - r.obj) <= 1e-12 * max(1, abs(r.obj))
        ht = np.concatenate([h, np.zeros(e, np.uint32)])
        rt = oracle.search(ht, k, q, mode, lib=lib)
        assert rt.thr.tolist() == r.thr.tolist() and abs(rt.obj - r.obj) <= 1e-12 * max(1, abs(r.obj))


def pin_direct_vs_prefix(lib=None):
    rng = np.random.default_rng(23)
    for trial in range(30):
        L = int(rng.integers(3, 17))
        k = int(rng.integers(1, min(3, L - 1) + 1))
        q = float(rng.choice([0.3, 0.5, 0.8, 1.2, 1.5, 2.0, 3.0]))
        h = rng.integers(0, 9, L).astype(np.uint32)
        h[rng.random(L) < 0.3] = 0
        d = oracle.search(h, k, q, oracle.MODE_DIRECT, lib=lib)
        p = oracle.search(h, k, q, oracle.MODE_PREFIX, lib=lib)
        assert d.status == p.status, (h, k, q, d, p)
        if d.status != oracle.OK:
            continue
        assert abs(d.obj - p.obj) <= 1e-12 * max(1, abs(d.obj)), (h, k, q, d, p)
        if d.thr.tolist() != p.thr.tolist():
            assert d.rel_gap() < 1e-12, (h, k, q, d, p)
        for t in _tuples(L, k):
            a = oracle.objective(h, t, q, oracle.MODE_DIRECT, lib=lib)
            b = oracle.objective(h, t, q, oracle.MODE_PREFIX, lib=lib)
            assert (np.isnan(a) and np.isnan(b)) or abs(a - b) <= 1e-12 * max(1, abs(a)), (h, t, q, a, b)


def pin_prefix(lib=None):
    rng = np.random.default_rng(29)
    h = rng.integers(0, 50, 64).astype(np.uint32)
    h[[5, 6, 7, 30, 63]] = 0
    for q in (0.5, 0.8, 1.5):
        P, Q = oracle.prefix(h, q, lib=lib)
        assert P[-1] == 1.0
        assert np.all(np.diff(P) >= 0) and np.all(np.diff(Q) >= 0)
        z = np.nonzero(h == 0)[0]
        z = z[z > 0]
        assert np.array_equal(P[z], P[z - 1]) and np.array_equal(Q[z], Q[z - 1]), "empty bins must repeat the prefix bit for bit"
        p = h / h.sum()
        assert abs(Q[-1] - np.sum(p[p > 0] ** q)) <= 1e-13 * Q[-1]
        C = np.cumsum(h.astype(np.int64))
        assert np.array_equal(P, C / C[-1])
    # uniform: Q(L-1) = L * L^-q
    P, Q = oracle.prefix(np.ones(32, np.uint32), 0.5, lib=lib)
    assert abs(Q[-1] - 32 * 32 ** -0.5) <= 1e-13


def pin_labels(lib=None):
    rng = np.random.default_rng(31)
    v = rng.integers(-1200, 3200, 3000).astype(np.int16)
    for lo, hi, L in WINDOWS[:5]:
        b = edge_bins(v, lo, hi, L)
        for k in (1, 2, 3):
            thr = np.sort(rng.choice(L - 1, k, replace=False)).astype(np.int32)
            lab = oracle.label(v, lo, hi, L, thr, lib=lib)
            assert np.array_equal(lab, np.searchsorted(thr, b, side="left").astype(np.uint8)), (lo, hi, L, thr)
        # Algorithm 1 with one threshold: foreground iff bin >= T, T = t + 1
        t = int(rng.integers(0, L - 1))
        lab = oracle.label(v, lo, hi, L, [t], lib=lib)
        assert np.array_equal(lab, (b >= t + 1).astype(np.uint8))
    assert not oracle.label(v, -1024, 3071, 4096, [-1], lib=lib).any(), "no valid tuple labels everything 0"


# ---- the multilevel variant: sum_j S_j + (1-q) prod_j S_j ----------------

SP = oracle.COMP_SUMPROD


def _sumprod_closed(sizes, q):
    S = [ln_q(m, q) for m in sizes]
    return sum(S) + (1.0 - q) * float(np.prod(S))


def pin_sumprod_uniform_closed_form(lib=None, mode=oracle.MODE_PREFIX):
    """Uniform histogram: each class entropy is ln_q(m_j) (m_j bins), so the
    variant is sum ln_q(m_j) + (1-q) prod ln_q(m_j); the arg max is the first
    tuple whose class sizes maximise that closed form."""
    for L, k, q in [(10, 2, 0.5), (9, 3, 1.5), (12, 2, 2.0), (16, 3, 0.8), (8, 1, 0.7), (11, 2, 3.0)]:
        h = np.full(L, 3, dtype=np.uint32)
        best, best_t = -np.inf, None
        for t in _tuples(L, k):
            want = _sumprod_closed(_class_sizes(L, t), q)
            S = oracle.objective(h, t, q, mode, lib=lib, comp=SP)
            assert abs(S - want) <= 1e-12 * max(1.0, abs(want)), f"sumprod uniform L={L} k={k} q={q} t={t}"
            if want > best + 1e-12 * max(1.0, abs(want)):
                best, best_t = want, t
        r = oracle.search(h, k, q, mode, lib=lib, comp=SP)
        assert abs(r.obj - best) <= 1e-12 * max(1.0, abs(best)), (L, k, q, r, best)
        got = _sumprod_closed(_class_sizes(L, r.thr.tolist()), q)
        assert abs(got - best) <= 1e-12 * max(1.0, abs(best)), (L, k, q, r, best_t)


def pin_sumprod_k1_is_paper(lib=None, mode=oracle.MODE_PREFIX):
    """One threshold: both compositions are the paper's H1 + H2 + (1-q) H1 H2."""
    rng = np.random.default_rng(23)
    for q in (0.4, 0.9, 1.6, 2.5):
        h = rng.integers(0, 40, 19).astype(np.uint32)
        for t in range(18):
            a = oracle.objective(h, [t], q, mode, lib=lib)
            b = oracle.objective(h, [t], q, mode, lib=lib, comp=SP)
            assert (np.isnan(a) and np.isnan(b)) or abs(a - b) <= 1e-13 * max(1.0, abs(a)), (q, t, a, b)
        ra, rb = oracle.search(h, 1, q, mode, lib=lib), oracle.search(h, 1, q, mode, lib=lib, comp=SP)
        assert ra.thr.tolist() == rb.thr.tolist(), (q, ra, rb)


def _gini_classes(h, t):
    p = h / h.sum()
    edges = [-1] + list(t) + [len(h) - 1]
    out = []
    for j in range(len(t) + 1):
        c = p[edges[j] + 1: edges[j + 1] + 1]
        out.append(1.0 - float(np.sum((c / c.sum()) ** 2)))
    return out


def pin_sumprod_q2(lib=None, mode=oracle.MODE_PREFIX):
    """q = 2: class entropies are Gini-Simpson indices 1 - sum (p/w)^2, so
    the variant is sum G_j - prod G_j."""
    rng = np.random.default_rng(29)
    for L, k in [(9, 2), (8, 3)]:
        h = rng.integers(1, 50, L).astype(np.uint32)
        for t in _tuples(L, k):
            G = _gini_classes(h, t)
            want = sum(G) - float(np.prod(G))
            S = oracle.objective(h, t, 2.0, mode, lib=lib, comp=SP)
            assert abs(S - want) <= 1e-12, (L, k, t, S, want)


def pin_sumprod_kapur_limit(lib=None, mode=oracle.MODE_PREFIX):
    """q -> 1: the product term vanishes and the variant tends to the sum of
    the class Shannon entropies."""
    rng = np.random.default_rng(31)
    for L, k in [(10, 2), (9, 3)]:
        h = rng.integers(1, 200, L).astype(np.uint32)
        for t in _tuples(L, k):
            K = _kapur(h, t)
            for q in (1.0 - 1e-6, 1.0 + 1e-6):
                S = oracle.objective(h, t, q, mode, lib=lib, comp=SP)
                assert abs(S - K) <= 1e-5 * (1.0 + K) ** 3, (L, k, t, q, S, K)


def pin_sumprod_symmetry(lib=None, mode=oracle.MODE_PREFIX):
    rng = np.random.default_rng(37)
    for L, k, q in [(14, 2, 0.5), (12, 3, 1.5)]:
        half = rng.integers(0, 30, L // 2).astype(np.uint32)
        h = np.concatenate([half, half[::-1]])
        for t in _tuples(L, k):
            mt = tuple(sorted(L - 2 - x for x in t))
            a = oracle.objective(h, t, q, mode, lib=lib, comp=SP)
            b = oracle.objective(h, mt, q, mode, lib=lib, comp=SP)
            assert (np.isnan(a) and np.isnan(b)) or abs(a - b) <= 1e-12 * max(1, abs(a)), (t, mt, a, b)


ALL_PINS = [
    pin_binmap_identity, pin_binmap_edges, pin_histogram, pin_uniform_closed_form, pin_uniform_argmax,
    pin_separated_bins, pin_q2_gini_simpson, pin_kapur_limit, pin_dp, pin_search_dp, pin_symmetry, pin_invariances,
    pin_direct_vs_prefix, pin_prefix, pin_labels, pin_sumprod_uniform_closed_form, pin_sumprod_k1_is_paper,
    pin_sumprod_q2, pin_sumprod_kapur_limit, pin_sumprod_symmetry,
]
MODE_PINS = [pin_uniform_closed_form, pin_uniform_argmax, pin_separated_bins, pin_q2_gini_simpson,
             pin_kapur_limit, pin_dp, pin_symmetry, pin_invariances, pin_sumprod_uniform_closed_form,
             pin_sumprod_k1_is_paper, pin_sumprod_q2, pin_sumprod_kapur_limit, pin_sumprod_symmetry]
