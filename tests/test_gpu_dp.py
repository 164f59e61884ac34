"""GPU parity of the dynamic-programming search (ts_threshold_search_dp):
against the exhaustive oracle for k up to 6 on small histograms (thresholds
identical unless the oracle's best two objectives are within 1e-6, objective
within 1e-5 relative), edge cases and exact ties (the first tuple), batched
q, and k = 4 on the 1024-level workload histogram (too many tuples for the
exhaustive oracle: the maximum is checked against an independent numpy
dynamic programme over the product identity, and the tuple against the
oracle's objective)."""
import numpy as np
import pytest

import oracle
from gpu_util import check_choice, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2012_10684_amd import api, synth  # noqa: E402


def _omode(q):
    return oracle.MODE_KAPUR if q == 1.0 else oracle.MODE_DIRECT


def _dp(H, k, q):
    P, Q = api.prefix(to_dev(H.view(np.int32)), q)
    thr, obj, st = api.threshold_search_dp(P, Q, k, q)
    torch.cuda.synchronize()
    return thr.cpu().numpy(), obj.cpu().numpy(), st.cpu().numpy()


def _random_hists(rng, n, L, zero_frac=0.3, hi=50):
    H = rng.integers(0, hi, (n, L)).astype(np.uint32)
    H[rng.random((n, L)) < zero_frac] = 0
    return H


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("q", [0.3, 0.8, 1.0, 1.5, 3.0])
def test_dp_small_random(k, q):
    rng = np.random.default_rng(700 * k + int(q * 10))
    for L in (k + 1, k + 2, 13, 24):
        H = _random_hists(rng, 4, L)
        thr, obj, st = _dp(H, k, q)
        for i in range(len(H)):
            check_choice(H[i], k, q, thr[i], obj[i], st[i], mode=_omode(q))


def test_dp_edge_cases():
    L = 30
    cases = [np.zeros(L, np.uint32)]
    one = np.zeros(L, np.uint32)
    one[11] = 9
    cases.append(one)
    for occ in ([0, 29], [3, 4, 20], [1, 2, 3, 28], [0, 5, 6, 13, 14, 29]):
        h = np.zeros(L, np.uint32)
        h[occ] = 5
        cases.append(h)
    cases.append(np.full(L, 3, np.uint32))
    half = np.arange(1, L // 2 + 1, dtype=np.uint32)
    cases.append(np.concatenate([half, half[::-1]]))
    H = np.stack(cases)
    for k in (1, 2, 3, 5):
        for q in (0.5, 1.5):
            thr, obj, st = _dp(H, k, q)
            for i in range(len(H)):
                check_choice(H[i], k, q, thr[i], obj[i], st[i], mode=oracle.MODE_DIRECT)


def test_dp_exact_ties_first_tuple():
    L = 48
    h = np.zeros(L, np.uint32)
    h[[2, 3, 15, 16, 17, 30, 31, 40, 46]] = [5, 9, 4, 4, 7, 3, 8, 2, 6]
    for k in (1, 2, 3, 4):
        thr, obj, st = _dp(h[None], k, 0.8)
        r = oracle.search(h, k, 0.8, oracle.MODE_DIRECT)
        assert thr[0].tolist() == r.thr.tolist(), (k, thr[0], r)


def test_dp_matches_exhaustive_on_workload_slices():
    """k = 1..3 on slices of the 300-slice workload: the same tuples as the
    oracle's exhaustive search."""
    vol = synth.workload_volume300(0)[::100]
    binn = api.binning(-1024, -200, 256)
    h = api.histogram(api.Batch.slices(to_dev(vol)), binn)
    torch.cuda.synchronize()
    H = h.cpu().numpy().view(np.uint32)
    for k in (1, 2, 3):
        for q in (0.5, 1.5):
            thr, obj, st = _dp(H, k, q)
            for i in range(len(H)):
                check_choice(H[i], k, q, thr[i], obj[i], st[i], mode=oracle.MODE_PREFIX)


def test_dp_batched_q_equals_single_calls():
    rng = np.random.default_rng(47)
    H = _random_hists(rng, 6, 120)
    Hd = to_dev(H.view(np.int32))
    qs = (0.5, 1.0, 2.0)
    P, Q = api.prefix(Hd, qs)
    thr, obj, st = api.threshold_search_dp(P, Q, 4, qs)
    for j, q in enumerate(qs):
        P1, Q1 = api.prefix(Hd, q)
        t1, o1, s1 = api.threshold_search_dp(P1, Q1, 4, q)
        assert torch.equal(thr[j], t1) and torch.equal(st[j], s1)
        assert np.array_equal(obj[j].cpu().numpy(), o1.cpu().numpy(), equal_nan=True)


def _numpy_dp_max(h, k, q):
    """max over tuples of sum_j sgn(1-q) [ln sum c^q - q ln C] (N cancels), by a
    vectorised dynamic programme over the last class boundary; returns S."""
    c = h.astype(np.float64)
    L = len(c)
    C = np.concatenate([[0.0], np.cumsum(c)])
    X = np.concatenate([[0.0], np.cumsum(np.where(c > 0, c ** q, 0.0))])
    s = 1.0 if q < 1 else -1.0

    def term(a, b):  # classes a..b for a vector of a and one b
        w = C[b + 1] - C[a]
        x = X[b + 1] - X[a]
        with np.errstate(divide="ignore", invalid="ignore"):
            t = s * (np.log(x) - q * np.log(w))
        return np.where(w > 0, t, -np.inf)

    best = np.array([term(np.array([0]), b)[0] for b in range(L)])  # one class 0..b
    for _ in range(k):
        nxt = np.full(L, -np.inf)
        for b in range(1, L):
            a = np.arange(1, b + 1)
            nxt[b] = np.max(best[a - 1] + term(a, b))
        best = nxt
    return np.expm1(s * best[L - 1]) / (1.0 - q)


@pytest.mark.parametrize("q", [0.8, 1.5])
def test_dp_k4_whole_volume_histogram(q):
    """k = 4 over the 1024-level histogram of a 512x512x120 volume
    (C(1023, 4) = 4.5e10 tuples)."""
    vol = synth.make_volume(synth.rng_for(3, 0), 120, 512)
    binn = api.binning(-1024, 3071, 1024)
    h = api.histogram(api.Batch([to_dev(vol).reshape(-1)]), binn)
    torch.cuda.synchronize()
    H = h.cpu().numpy().view(np.uint32)
    thr, obj, st = _dp(H, 4, q)
    assert st[0] == 0
    # the oracle's own dynamic programme (pinned against the exhaustive
    # oracle and an independent numpy programme): same tuple, same value
    r = oracle.search_dp(H[0], 4, q)
    assert r.status == oracle.OK
    assert abs(obj[0] - r.obj) <= 1e-9 * abs(r.obj), (obj[0], r)
    s_or = oracle.objective(H[0], thr[0], q, oracle.MODE_PREFIX)
    assert abs(s_or - r.obj) <= 1e-9 * abs(r.obj), (thr[0], s_or, r)
    if thr[0].tolist() != r.thr.tolist():  # only a tie within FP64 rounding may differ
        assert abs(s_or - r.obj) <= 1e-12 * abs(r.obj), (thr[0].tolist(), r)
    want = _numpy_dp_max(H[0], 4, q)
    assert abs(obj[0] - want) <= 1e-9 * abs(want), (obj[0], want)
    # the four thresholds label the volume (labels 0..4)
    dv = to_dev(vol).reshape(-1)
    lab = api.label(api.Batch([dv]), binn, to_dev(thr), 4)[0]
    torch.cuda.synchronize()
    assert np.array_equal(lab.cpu().numpy(), oracle.label(vol.reshape(-1), -1024, 3071, 1024, thr[0]))
    say(f"k=4 q={q}: thresholds {thr[0].tolist()} S={obj[0]!r}")
