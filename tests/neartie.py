"""Adversarial near-tie histograms for the precision tests (FP32 keys against
the FP64 arg max).  Built with the oracle only.

Every case is a histogram plus two threshold tuples, `first` and `later`
(first < later lexicographically), such that the oracle's arg max is `later`,
its runner-up is `first`, and the two objectives differ by a relative amount
between 1e-13 and 1e-8.  That gap is far above FP64 rounding but below what
FP32 keys resolve, and when the two FP32 keys come out equal the first-tuple
rule picks `first`.  An FP32-only search therefore often returns `first`, and
an exact search must return `later`.

Two constructions:
  mirror    a mirror-symmetric histogram (c_i = c_{L-1-i}) whose optimum is
            not its own mirror image, so tuple and mirror tie exactly; then one
            count is perturbed by a few units out of ~1e7, which breaks the tie
            in favour of the mirror (the later tuple);
  tiny_bin  a histogram of counts ~1e6-1e7 in which one bin holds only a few
            counts; moving one threshold of the optimum across that bin changes
            the class masses by ~1e-9 relative, and the case keeps the
            direction in which the later tuple wins.
"""
from __future__ import annotations

import numpy as np

import oracle

GAP_MIN, GAP_MAX = 1e-13, 1e-8


def mirror_of(t, L):
    return sorted(L - 2 - x for x in t)


def _accept(h, k, q, first, later):
    r = oracle.search(h, k, q)
    if r.status != oracle.OK or r.thr.tolist() != later:
        return None
    s_first = oracle.objective(h, first, q)
    gap = (r.obj - s_first) / abs(r.obj)
    # the runner-up over every tuple must be `first` itself
    if not (GAP_MIN <= gap <= GAP_MAX) or r.rel_gap() != gap:
        return None
    return gap


def mirror_case(rng, L, k, q, base=1e7, tries=200):
    for _ in range(tries):
        half = rng.uniform(0.2, 1.0, L // 2) ** rng.uniform(1, 4)
        h = np.round(np.concatenate([half, half[::-1]]) * base).astype(np.uint32)
        r = oracle.search(h, k, q)
        t = r.thr.tolist()
        first, later = sorted([t, mirror_of(t, L)])
        if later == first:
            continue  # self-mirror optimum: no pair to split
        for j in rng.permutation(L):
            for d in (1, 2, 3, 5, 8, 13, 21, 34, 55, 89):
                done = False
                for sgn in (1, -1):
                    h2 = h.copy()
                    h2[j] = np.uint32(int(h2[j]) + sgn * d)
                    if oracle.search(h2, k, q).thr.tolist() != later:
                        continue
                    gap = _accept(h2, k, q, first, later)
                    if gap is not None:
                        return dict(hist=h2, first=first, later=later, gap=gap, kind="mirror", sym=h)
                    done = True  # the perturbation is already too large on this bin
                    break
                if done:
                    break
    return None


def tiny_bin_case(rng, L, k, q, small, tries=100):
    for _ in range(tries):
        h = np.round(rng.uniform(1e6, 1e7, L) * rng.uniform(0.2, 1.0, L) ** 2).astype(np.uint32)
        t = oracle.search(h, k, q).thr.tolist()
        for j in rng.permutation(k):
            for b in (t[j] + 1, t[j]):  # the bin that threshold j moves across
                prev = t[j - 1] if j else -1
                nxt = t[j + 1] if j + 1 < k else L - 1
                if b - 1 <= prev or b >= nxt or b > L - 2:
                    continue
                h2 = h.copy()
                h2[b] = small
                first, later = list(t), list(t)
                first[j], later[j] = b - 1, b
                gap = _accept(h2, k, q, first, later)
                if gap is not None:
                    return dict(hist=h2, first=first, later=later, gap=gap, kind="tiny_bin", sym=None)
    return None


# (q, counts in the tiny bin).  For q > 1 the tiny bin is kept large enough
# that the smallest class sum stays within the range the FP32 error bound
# covers.  For q = 0.5 there is no tiny-bin case: one count adds p^0.5 ~ 6e-5
# of a class sum of ~8, a gap far above FP32 resolution.
TINY = ((0.5, None), (0.8, 1), (1.5, 8), (2.0, 256))
QS = tuple(q for q, _ in TINY)
LEVELS = {"mirror": (32, 32, 24), "tiny_bin": (64, 64, 40)}  # L for k = 1, 2, 3


def cases(k: int, q: float, n_mirror: int = 4, n_tiny: int = 4, seed: int = 0):
    """Near-tie cases for k thresholds at index q: up to n_mirror mirror cases
    (L = 32 for k <= 2, 24 for k = 3) and n_tiny tiny-bin cases (L = 64 or
    40); twice as many mirror cases where q has no tiny-bin case."""
    rng = np.random.default_rng([20121068, 7, k, int(q * 100), seed])
    small = dict(TINY)[q]
    out = []
    for _ in range(n_mirror if small else 2 * n_mirror):
        c = mirror_case(rng, LEVELS["mirror"][k - 1], k, q)
        if c is not None:
            out.append(c)
    for _ in range(n_tiny if small else 0):
        c = tiny_bin_case(rng, LEVELS["tiny_bin"][k - 1], k, q, small)
        if c is not None:
            out.append(c)
    return out
