"""The scratch-free search entry point (ts_threshold_search_noalloc) against
ts_threshold_search with a caller workspace: the same kernels, so the
thresholds, FP64 objectives and statuses must be identical bit for bit.
Two calls in a row on each search path that uses scratch, the second on a
smaller input, so stale contents left in the shared scratch by the first
call cannot leak into the second; the default one-workgroup path (no scratch)
and the oracle's thresholds on the second call as well; sizes beyond the
fixed scratch rejected before any launch."""
import numpy as np
import pytest

import oracle
from gpu_util import check_choice, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2012_10684_amd import api, synth  # noqa: E402


@pytest.fixture(scope="module")
def slices():
    return synth.make_volume(synth.rng_for(5, 11), 12, 256)


def _hists(vol, nz, lo, hi, L):
    return np.stack([oracle.histogram(vol[z], lo, hi, L) for z in range(nz)])


def _both(H, k, qs, path):
    hist = to_dev(H.view(np.int32))
    P, Q = api.prefix(hist, qs)
    tune = {"search_path": path} if path else None
    a = api.threshold_search(P, Q, k, qs, tune=tune)
    b = api.threshold_search_noalloc(P, Q, k, qs, tune=tune)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in a], [x.cpu().numpy() for x in b]


# (k, window, bins, path, problems of the first call, of the second)
CASES = [
    (3, (-1024, 3071), 1024, 0, 3, 1),    # k = 3 row kernels (scratch)
    (2, (-1024, -200), 256, 2, 12, 5),   # k = 2, one launch per phase (scratch)
    (1, (-1024, 3071), 1000, 2, 8, 3),   # k = 1, one launch per phase (scratch)
    (2, (-1024, -200), 256, 1, 12, 4),   # one workgroup per problem (no scratch)
]


@pytest.mark.parametrize("k,win,L,path,n1,n2", CASES, ids=["k3L1024", "k2L256tiled", "k1L1000tiled", "k2fused"])
def test_noalloc_equals_workspace_search(slices, k, win, L, path, n1, n2):
    qs = [0.5, 0.8, 1.5]
    for n in (n1, n2):
        say(f"noalloc: k={k} L={L} path={path} problems={n}")
        H = _hists(slices, n, win[0], win[1], L)
        (ta, oa, sa), (tb, ob, sb) = _both(H, k, qs, path)
        assert np.array_equal(ta, tb), (ta, tb)
        assert np.array_equal(oa.view(np.int64), ob.view(np.int64)), (oa, ob)
        assert np.array_equal(sa, sb)
        if n == n2:
            for j, q in enumerate(qs):
                for z in range(n):
                    check_choice(H[z], k, q, tb[j][z], ob[j][z], sb[j][z])


def test_noalloc_rejects_sizes_beyond_the_scratch():
    # k = 2 on 256 bins, one launch per phase, 20,000 problems: far more than
    # the fixed scratch; rejected on the host, nothing launched
    n, L = 20000, 256
    P = torch.zeros((n, L), dtype=torch.float64, device="cuda:0")
    Q = torch.zeros_like(P)
    with pytest.raises(api.TsError) as e:
        api.threshold_search_noalloc(P, Q, 2, 0.8, tune={"search_path": 2})
    assert e.value.status == 3 and "scratch" in str(e.value), e.value
    torch.cuda.synchronize()
