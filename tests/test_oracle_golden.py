"""The oracle against the stored closed-form values (tests/golden)."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "uniform_closed_form.txt")


def _rows():
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            L, k, q, t, S = line.split()
            yield int(L), int(k), float(q), [int(x) for x in t.split(",")], float(S)


@pytest.mark.parametrize("mode", [oracle.MODE_DIRECT, oracle.MODE_PREFIX], ids=["direct", "prefix"])
def test_uniform_closed_form_golden(mode):
    rows = list(_rows())
    assert len(rows) > 50
    for L, k, q, t, S in rows:
        got = oracle.objective(np.full(L, 5, np.uint32), t, q, mode)
        assert abs(got - S) <= 2e-15 * max(1.0, abs(S)) * L, (L, k, q, t, got, S)
