"""Helpers shared by the GPU parity tests: upload seeded inputs, run the HIP
path through the binding, and compare with the oracle under the acceptance
rule (thresholds identical unless the oracle's runner-up is within 1e-6
relative of its optimum; objective within 1e-5 relative)."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle

THR_REL_TIE = 1e-6
OBJ_REL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev():
    return torch.device("cuda:0")


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def check_choice(h: np.ndarray, k: int, q: float, thr, obj, status, mode=oracle.MODE_PREFIX, ref=None,
                 comp=oracle.COMP_RECURSIVE):
    """Compare one GPU search result with the oracle (objective composed as
    comp).  Returns (exact, ref)."""
    r = ref if ref is not None else oracle.search(h, k, q, mode, comp=comp)
    thr = [int(x) for x in np.asarray(thr).reshape(-1)]
    if r.status != oracle.OK:
        assert status == r.status, (status, r)
        assert thr == [-1] * k, thr
        assert np.isnan(obj), obj
        return True, r
    assert status == 0, (status, r)
    exact = thr == r.thr.tolist()
    if not exact:
        s_gpu = oracle.objective(h, thr, q, mode, comp=comp)
        assert np.isfinite(s_gpu), (thr, r)
        assert s_gpu >= r.obj - THR_REL_TIE * abs(r.obj), (
            f"thresholds {thr} vs oracle {r.thr.tolist()}: S {s_gpu!r} vs {r.obj!r} (gap {r.rel_gap():.3g})")
    tol = OBJ_REL * abs(r.obj) + 1e-12
    assert abs(obj - r.obj) <= tol, (obj, r.obj, thr, r)
    return exact, r
