"""The adversarial near-tie cases of the precision tests, checked on the CPU:
the oracle's arg max is the later tuple, its runner-up is the earlier one, the
gap lies between FP64 rounding and FP32 resolution, the oracle's literal-sum
mode agrees on the choice, and the constructions do what they claim (mirror
symmetry before the perturbation; one threshold moved across a nearly empty
bin)."""
import numpy as np
import pytest

import oracle
from neartie import GAP_MAX, GAP_MIN, QS, TINY, cases, mirror_of


@pytest.mark.parametrize("q", QS)
@pytest.mark.parametrize("k", [1, 2, 3])
def test_near_tie_cases(k, q):
    cs = cases(k, q)
    assert len(cs) >= 4, (k, q, len(cs))
    assert {c["kind"] for c in cs} == ({"mirror", "tiny_bin"} if dict(TINY)[q] else {"mirror"}), (k, q)
    for c in cs:
        h, first, later = c["hist"], c["first"], c["later"]
        L = h.size
        assert first < later and len(first) == k
        r = oracle.search(h, k, q)
        assert r.thr.tolist() == later
        assert r.second == oracle.objective(h, first, q)
        assert GAP_MIN <= r.rel_gap() <= GAP_MAX, r.rel_gap()
        # the literal class sums pick the same tuple
        assert oracle.search(h, k, q, oracle.MODE_DIRECT).thr.tolist() == later
        if c["kind"] == "mirror":
            sym = c["sym"]
            assert np.array_equal(sym, sym[::-1])
            assert mirror_of(first, L) == later
            s1, s2 = oracle.objective(sym, first, q), oracle.objective(sym, later, q)
            assert abs(s1 - s2) <= 1e-13 * abs(s1)
            assert int(np.abs(h.astype(np.int64) - sym).sum()) <= 89
            # the pair ties up to FP64 rounding before the perturbation
            assert oracle.search(sym, k, q).thr.tolist() in (first, later)
        else:
            moved = [j for j in range(k) if first[j] != later[j]]
            assert len(moved) == 1
            j = moved[0]
            assert later[j] == first[j] + 1
            assert int(h[later[j]]) == dict(TINY)[q]
