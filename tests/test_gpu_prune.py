"""Row pruning of the k = 2 one-workgroup search: rows whose upper bound
(head term + a bound on the middle class term + the block's largest tail
term) falls below a seed key by three error bounds are skipped in phase 1.
The result must not change: on histograms of many shapes the one-workgroup
path (pruned) returns the same thresholds and the same FP64 objective bits
as the one-launch-per-phase path (every row evaluated), and the oracle's
tuple."""
import numpy as np
import pytest

import oracle
from gpu_util import check_choice, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2012_10684_amd import api, synth  # noqa: E402

QS = [0.3, 0.8, 1.0, 1.5, 3.0]


def _shapes(L, seed):
    """Histograms of L bins: mixtures of bumps, sparse spikes, flat noise,
    geometric decay, runs of empty bins, a CT-like slice's levels."""
    rng = np.random.default_rng(seed)
    x = np.arange(L)
    out = []
    for _ in range(3):
        h = np.zeros(L)
        for _ in range(rng.integers(1, 5)):
            c, w = rng.uniform(0, L), rng.uniform(0.5, L / 4 + 1)
            h += rng.uniform(1e3, 1e6) * np.exp(-0.5 * ((x - c) / w) ** 2)
        out.append(h)
    h = np.zeros(L)
    h[rng.choice(L, size=max(2, L // 10), replace=False)] = rng.integers(1, 10 ** 6, size=max(2, L // 10))
    out.append(h)
    out.append(rng.integers(0, 1000, size=L).astype(float))
    out.append(1e6 * 0.97 ** x)
    h = rng.integers(0, 5000, size=L).astype(float)
    h[rng.integers(0, L):][: rng.integers(1, L)] = 0
    out.append(h)
    return [np.floor(v).astype(np.uint32) for v in out]


def _run(H, q, path):
    P, Q = api.prefix(to_dev(H.view(np.int32)), q)
    thr, obj, st = api.threshold_search(P, Q, 2, q, api.SEARCH_FP32_TIECHECK, tune={"search_path": path})
    torch.cuda.synchronize()
    return thr.cpu().numpy(), obj.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("L", [3, 4, 17, 64, 65, 200, 256, 300, 1000, 1024])
def test_pruned_equals_unpruned_and_oracle(L):
    H = np.stack(_shapes(L, 1000 + L))
    for q in QS:
        say(f"k=2 pruning L={L} q={q}: {H.shape[0]} histograms")
        t1, o1, s1 = _run(H, q, 1)  # one workgroup per problem (pruned)
        t2, o2, s2 = _run(H, q, 2)  # one launch per phase (every row)
        assert np.array_equal(t1, t2), (q, t1, t2)
        assert np.array_equal(o1.view(np.int64), o2.view(np.int64)), (q, o1, o2)
        assert np.array_equal(s1, s2)
        mode = oracle.MODE_KAPUR if q == 1.0 else oracle.MODE_PREFIX
        for i in range(H.shape[0]):
            check_choice(H[i], 2, q, t1[i], o1[i], s1[i], mode=mode)


def test_pruned_on_ct_slices():
    vol = synth.workload_volume300(0)[::25]
    H = np.stack([oracle.histogram(z, -1024, -200, 256) for z in vol]).astype(np.uint32)
    for q in (0.5, 0.8, 1.5):
        say(f"k=2 pruning on {H.shape[0]} CT slices, q={q}")
        t1, o1, s1 = _run(H, q, 1)
        t2, o2, s2 = _run(H, q, 2)
        assert np.array_equal(t1, t2) and np.array_equal(o1.view(np.int64), o2.view(np.int64))
        for i in range(H.shape[0]):
            exact, _ = check_choice(H[i], 2, q, t1[i], o1[i], s1[i])
            assert exact


@pytest.mark.parametrize("L", [4, 5, 17, 64, 65, 200, 300])
def test_k3_group_pruning(L):
    """k = 3: k_rows3 skips row groups whose bound (largest A of the group +
    largest column term) is below the seeds' threshold; the thresholds must
    equal those of the FP64 exhaustive mode (no pruning) and the oracle's."""
    H = np.stack(_shapes(L, 3000 + L))
    for q in QS:
        say(f"k=3 pruning L={L} q={q}: {H.shape[0]} histograms")
        P, Q = api.prefix(to_dev(H.view(np.int32)), q)
        t1, o1, s1 = (x.cpu().numpy() for x in api.threshold_search(P, Q, 3, q, api.SEARCH_FP32_TIECHECK))
        t2, o2, s2 = (x.cpu().numpy() for x in api.threshold_search(P, Q, 3, q, api.SEARCH_FP64))
        torch.cuda.synchronize()
        assert np.array_equal(t1, t2), (q, t1, t2)
        assert np.array_equal(s1, s2)
        mode = oracle.MODE_KAPUR if q == 1.0 else oracle.MODE_PREFIX
        for i in range(H.shape[0]):
            check_choice(H[i], 3, q, t1[i], o1[i], s1[i], mode=mode)
