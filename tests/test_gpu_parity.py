"""GPU parity of every step of the path against the CPU oracle, element by
element on seeded inputs: histograms and labels bit-exact, P bit-exact, Q to
summation-order rounding, thresholds identical (up to the stated tie rule) and
objectives within 1e-5 relative.  Sizes span several tiles with ragged tails;
edge cases cover empty, one-voxel and unaligned problems, degenerate
histograms, exact ties and narrow windows."""
import numpy as np
import pytest

import oracle
from gpu_util import check_choice, say, to_dev, u32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2012_10684_amd import api, synth  # noqa: E402

WINDOWS = [(-1024, 3071, 4096), (-1024, 3071, 1024), (-1024, -200, 256), (-1024, 3071, 512),
           (-5, 7, 13), (100, 100, 4), (-32768, 32767, 4096), (3, 1000, 7), (-1024, -1000, 256)]
MODES = [api.SEARCH_FP32_TIECHECK, api.SEARCH_FP64, api.SEARCH_PLAIN]


def ragged_segments(rng, base: torch.Tensor):
    """Views of one buffer at assorted offsets and lengths (incl. empty,
    one voxel, unaligned starts, lengths not a multiple of 8)."""
    sizes = [0, 1, 7, 8, 9, 63, 1000, 4097, 65537, 0, 3, 262144]
    segs, pos = [], 0
    for n in sizes:
        pos += int(rng.integers(0, 9))  # misalign the start
        segs.append(base[pos:pos + n])
        pos += n
    return segs


@pytest.fixture(scope="module")
def ragged():
    rng = np.random.default_rng(101)
    host = synth.make_volume(synth.rng_for(9, 1), 2, 512).reshape(-1)[:400000].copy()
    host[:50] = np.arange(-32768, 32767, 1311)[:50]  # extreme values
    base = to_dev(host)
    segs = ragged_segments(rng, base)
    return host, base, segs


@pytest.mark.parametrize("win", WINDOWS, ids=lambda w: f"{w[0]}_{w[1]}_{w[2]}")
def test_histogram_ragged_batch(ragged, win):
    host, base, segs = ragged
    lo, hi, L = win
    b = api.Batch(segs)
    h = u32(api.histogram(b, api.binning(lo, hi, L)))
    torch.cuda.synchronize()
    for i, s in enumerate(segs):
        want = oracle.histogram(s.cpu().numpy(), lo, hi, L)
        assert np.array_equal(h[i], want), (win, i, s.numel())
        assert int(h[i].sum()) == s.numel()


@pytest.mark.parametrize("win", WINDOWS, ids=lambda w: f"{w[0]}_{w[1]}_{w[2]}")
def test_histogram_every_int16(win):
    lo, hi, L = win
    allv = np.arange(-32768, 32768, dtype=np.int64).astype(np.int16)
    h = u32(api.histogram(api.Batch([to_dev(allv)]), api.binning(lo, hi, L)))[0]
    assert np.array_equal(h, oracle.histogram(allv, lo, hi, L)), win


@pytest.mark.parametrize("off", [0, 1, 2, 3])
@pytest.mark.parametrize("L", [13, 256])
def test_histogram_into_offset_view(ragged, off, L):
    """The output may start at any word: the zero fill's head, 16-byte body
    and tail all land in the histogram rows and nowhere else, over a buffer
    holding junk from an earlier use."""
    host, base, segs = ragged
    lo, hi = (-5, 7) if L == 13 else (-1024, -200)
    n = len(segs) * L
    buf = torch.full((n + 8,), 0x5EED, dtype=torch.int32, device=base.device)
    out = buf[off:off + n].view(len(segs), L)
    api.histogram(api.Batch(segs), api.binning(lo, hi, L), out=out)
    got = buf.cpu().numpy()
    assert np.all(got[:off] == 0x5EED) and np.all(got[off + n:] == 0x5EED), "words outside the rows changed"
    h = got[off:off + n].reshape(len(segs), L).view(np.uint32)
    for i, sg in enumerate(segs):
        assert np.array_equal(h[i], oracle.histogram(sg.cpu().numpy(), lo, hi, L)), (off, L, i)


@pytest.mark.parametrize("tune", [None, dict(hist_replicas=1, hist_block=64), dict(hist_replicas=4, hist_block=1024),
                                  dict(hist_wg_per_cu=1, min_chunk=512)], ids=["default", "r1b64", "r4b1024", "small"])
def test_histogram_tuning_invariant(ragged, tune):
    host, base, segs = ragged
    b = api.Batch(segs)
    binn = api.binning(-1024, -200, 256)
    ref = u32(api.histogram(b, binn))
    got = u32(api.histogram(b, binn, tune=tune))
    assert np.array_equal(ref, got)


def _prefix_case(rng, L):
    h = rng.integers(0, 1000, L).astype(np.uint32)
    h[rng.random(L) < 0.4] = 0
    return h


@pytest.mark.parametrize("q", [0.3, 0.8, 1.5, 2.5])
def test_prefix(q):
    rng = np.random.default_rng(7)
    hs = [_prefix_case(rng, 1024) for _ in range(5)]
    hs.append(np.zeros(1024, np.uint32))  # empty problem
    one = np.zeros(1024, np.uint32)
    one[512] = 7
    hs.append(one)
    H = np.stack(hs)
    P, Q = api.prefix(to_dev(H.view(np.int32)), q)
    P, Q = P.cpu().numpy(), Q.cpu().numpy()
    for i, h in enumerate(hs):
        Po, Qo = oracle.prefix(h, q)
        assert np.array_equal(P[i], Po), i  # one rounding of an exact count ratio
        tol = 1024 * 2.0 ** -52 * np.maximum(Qo, 1e-300)
        assert np.all(np.abs(Q[i] - Qo) <= tol), (i, np.max(np.abs(Q[i] - Qo) / np.maximum(Qo, 1e-300)))
        z = np.nonzero(h == 0)[0]
        z = z[z > 0]
        assert np.array_equal(Q[i][z], Q[i][z - 1]), "an empty bin must repeat Q bit for bit"
        if h.sum():
            assert P[i][-1] == 1.0


def _search_all(H: np.ndarray, k: int, q: float, mode: int, tune=None):
    P, Q = api.prefix(to_dev(H.view(np.int32)), q)
    thr, obj, st = api.threshold_search(P, Q, k, q, mode, tune=tune)
    torch.cuda.synchronize()
    return thr.cpu().numpy(), obj.cpu().numpy(), st.cpu().numpy()


def _random_hists(rng, n, L, zero_frac=0.3, hi=50):
    H = rng.integers(0, hi, (n, L)).astype(np.uint32)
    H[rng.random((n, L)) < zero_frac] = 0
    return H


@pytest.mark.parametrize("mode", MODES, ids=["fp32tie", "fp64", "plain"])
@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("q", [0.3, 0.8, 1.5, 3.0])
def test_search_small_random(mode, k, q):
    rng = np.random.default_rng(1000 * k + int(q * 10) + mode)
    for L in (k + 1, k + 2, 13, 64, 130):
        H = _random_hists(rng, 6, L)
        thr, obj, st = _search_all(H, k, q, mode)
        for i in range(len(H)):
            check_choice(H[i], k, q, thr[i], obj[i], st[i], mode=oracle.MODE_DIRECT)


@pytest.mark.parametrize("mode", MODES, ids=["fp32tie", "fp64", "plain"])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_search_shannon_limit_small_random(mode, k):
    """q = 1: Kapur's objective (sum of class Shannon entropies) against the
    oracle's literal-sum Kapur mode."""
    rng = np.random.default_rng(7000 + 10 * k + mode)
    for L in (k + 1, k + 2, 13, 64, 130):
        H = _random_hists(rng, 6, L)
        thr, obj, st = _search_all(H, k, 1.0, mode)
        for i in range(len(H)):
            check_choice(H[i], k, 1.0, thr[i], obj[i], st[i], mode=oracle.MODE_KAPUR)


def test_prefix_shannon_limit():
    """q = 1: Q(t) = sum_{i<=t} p_i ln p_i, empty bins repeating Q exactly."""
    rng = np.random.default_rng(17)
    hs = [_prefix_case(rng, 1024) for _ in range(4)] + [np.zeros(1024, np.uint32)]
    one = np.zeros(1024, np.uint32)
    one[300] = 5  # p = 1: p ln p = 0
    hs.append(one)
    H = np.stack(hs)
    P, Q = api.prefix(to_dev(H.view(np.int32)), 1.0)
    Q = Q.cpu().numpy()
    for i, h in enumerate(hs):
        N = h.sum()
        if N == 0:
            assert not Q[i].any()
            continue
        p = h.astype(np.float64) / N
        want = np.cumsum(np.where(p > 0, p * np.log(np.where(p > 0, p, 1.0)), 0.0))
        tol = 1024 * 2.0 ** -52 * np.maximum(np.abs(want), 1e-300) + 1e-300
        assert np.all(np.abs(Q[i] - want) <= tol * 4), i
        z = np.nonzero(h == 0)[0]
        z = z[z > 0]
        assert np.array_equal(Q[i][z], Q[i][z - 1])


def test_search_shannon_limit_workload_slices():
    """q = 1 on slices of the 300-slice workload (256 bins, k = 2): the
    thresholds agree with the oracle's Kapur mode."""
    vol = synth.workload_volume300(0)[::50]
    dv = to_dev(vol)
    b = api.Batch.slices(dv)
    binn = api.binning(-1024, -200, 256)
    P, Q = api.prefix(api.histogram(b, binn), 1.0)
    thr, obj, st = api.threshold_search(P, Q, 2, 1.0)
    thr, obj, st = thr.cpu().numpy(), obj.cpu().numpy(), st.cpu().numpy()
    for z in range(vol.shape[0]):
        h = oracle.histogram(vol[z], -1024, -200, 256)
        check_choice(h, 2, 1.0, thr[z], obj[z], st[z], mode=oracle.MODE_KAPUR)


@pytest.mark.parametrize("mode", MODES, ids=["fp32tie", "fp64", "plain"])
def test_search_edge_cases(mode):
    L = 40
    cases = []
    cases.append(np.zeros(L, np.uint32))  # empty
    one = np.zeros(L, np.uint32)
    one[17] = 9
    cases.append(one)  # one occupied bin: degenerate for every k
    for occ in ([0, 39], [3, 4, 30], [1, 2, 3, 38]):  # exactly k+1 occupied bins for k = 1, 2, 3
        h = np.zeros(L, np.uint32)
        h[occ] = 5
        cases.append(h)
    cases.append(np.full(L, 3, np.uint32))  # uniform: exact ties everywhere
    half = np.arange(1, L // 2 + 1, dtype=np.uint32)
    cases.append(np.concatenate([half, half[::-1]]))  # symmetric
    H = np.stack(cases)
    for k in (1, 2, 3):
        for q in (0.5, 1.5):
            thr, obj, st = _search_all(H, k, q, mode)
            for i in range(len(H)):
                check_choice(H[i], k, q, thr[i], obj[i], st[i], mode=oracle.MODE_DIRECT)


def test_search_exact_ties_first_tuple():
    # runs of empty bins: every tuple moving a threshold inside a run ties
    # exactly; the first in lexicographic order must win
    L = 64
    h = np.zeros(L, np.uint32)
    h[[2, 3, 20, 21, 22, 50, 51, 60]] = [5, 9, 4, 4, 7, 3, 8, 2]
    for k in (1, 2, 3):
        for mode in MODES:
            thr, obj, st = _search_all(h[None], k, 0.8, mode)
            r = oracle.search(h, k, 0.8, oracle.MODE_DIRECT)
            assert thr[0].tolist() == r.thr.tolist(), (k, mode, thr[0], r)


@pytest.mark.parametrize("tune", [dict(search_cols=1), dict(search_cols=4), dict(search_cols=2, search_rows=256)],
                         ids=["c1", "c4", "c2r256"])
def test_search_tuning_invariant(tune):
    rng = np.random.default_rng(5)
    for k in (1, 2, 3):
        H = _random_hists(rng, 5, 300, zero_frac=0.2, hi=5000)
        a = _search_all(H, k, 0.8, api.SEARCH_FP32_TIECHECK)
        b = _search_all(H, k, 0.8, api.SEARCH_FP32_TIECHECK, tune=tune)
        for x, y in zip(a, b):
            assert np.array_equal(x, y, equal_nan=True)


def test_search_fp32_only_mode_is_close():
    rng = np.random.default_rng(11)
    H = _random_hists(rng, 8, 256, zero_frac=0.1, hi=10000)
    thr, obj, st = _search_all(H, 2, 0.8, api.SEARCH_FP32_ONLY)
    for i in range(len(H)):
        r = oracle.search(H[i], 2, 0.8)
        s = oracle.objective(H[i], thr[i], 0.8)
        assert s >= r.obj - 1e-4 * abs(r.obj)  # FP32 keys: near-optimal, not necessarily exact
        assert abs(obj[i] - s) <= 1e-10 * abs(s)  # reported value is the FP64 objective of that tuple


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("q", [0.5, 1.0, 1.5])
def test_search_plain_fp32_mode_is_close(k, q):
    """The plain form in FP32 (one thread per tuple, every class term in
    FP32): near-optimal against the oracle, its reported objective the FP64
    value of its own tuple, and the statuses of the exact modes (an empty
    and a one-bin histogram included)."""
    rng = np.random.default_rng(31 + k + int(10 * q))
    L = {1: 300, 2: 130, 3: 40}[k]
    H = _random_hists(rng, 5, L, zero_frac=0.1, hi=10000)
    H[3] = 0
    H[4] = 0
    H[4][7] = 50
    thr, obj, st = _search_all(H, k, q, api.SEARCH_PLAIN_FP32)
    _, _, st_ref = _search_all(H, k, q, api.SEARCH_PLAIN)
    assert np.array_equal(st, st_ref), (st, st_ref)
    assert st[3] == api.PROBLEM_EMPTY and st[4] == api.PROBLEM_DEGENERATE
    om = oracle.MODE_KAPUR if q == 1.0 else oracle.MODE_PREFIX  # q = 1: the Shannon limit
    for i in range(3):
        r = oracle.search(H[i], k, q, mode=om)
        s = oracle.objective(H[i], thr[i], q, mode=om)
        assert s >= r.obj - 1e-4 * abs(r.obj), (k, q, i, thr[i], r.thr)
        assert abs(obj[i] - s) <= 1e-10 * abs(s), (k, q, i)


def test_label_ragged(ragged):
    host, base, segs = ragged
    rng = np.random.default_rng(3)
    for lo, hi, L in WINDOWS:
        for k in (1, 2, 3):
            thr = np.stack([np.sort(rng.choice(L - 1, k, replace=False)) for _ in segs]).astype(np.int32)
            thr[1] = -1  # degenerate row
            if len(segs) > 4 and k >= 2:
                thr[4, :2] = [5, 5]  # not strictly ascending: labels 0
            b = api.Batch(segs)
            outs = api.label(b, api.binning(lo, hi, L), to_dev(thr), k)
            torch.cuda.synchronize()
            for i, s in enumerate(segs):
                want = oracle.label(s.cpu().numpy(), lo, hi, L, thr[i])
                if i == 4 and k >= 2:
                    want = np.zeros_like(want)
                assert np.array_equal(outs[i].cpu().numpy(), want), (lo, hi, L, k, i)


@pytest.mark.parametrize("win", [(32760, 32767, 16), (-32768, -32760, 16), (-32768, 32767, 4096), (32767, 32767, 4),
                                 (-32768, -32768, 5), (-1024, -200, 256)], ids=lambda w: f"{w[0]}_{w[1]}_{w[2]}")
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_label_every_int16(win, k):
    """Every int16 value, shuffled, in problems whose lengths are and are not
    multiples of 8: windows at both ends of the int16 range (cut values of
    -32767 and of 32768, the latter reached by no voxel), one and three
    threshold sets, thresholds including 0 and L - 2."""
    lo, hi, L = win
    if L - 1 < k:
        pytest.skip("fewer than k + 1 bins")
    rng = np.random.default_rng(k * 1000 + L)
    allv = rng.permutation(np.arange(-32768, 32768, dtype=np.int64).astype(np.int16))
    cuts = [0, 8192, 8195, 40000, 65536]  # problems of 8192, 3, 31805 and 25536 voxels
    segs = [allv[a:b] for a, b in zip(cuts[:-1], cuts[1:])]
    dsegs = [to_dev(sg) for sg in segs]
    thrs = []
    for u in range(3):
        rows = [np.sort(rng.choice(L - 1, k, replace=False)) for _ in segs]
        rows[u % len(segs)][0] = 0
        rows[(u + 1) % len(segs)][-1] = L - 2
        for r in rows:
            r.sort()
        thrs.append(np.stack(rows).astype(np.int32))
    b = api.Batch(dsegs)
    binn = api.binning(lo, hi, L)
    one = api.label(b, binn, to_dev(thrs[0]), k)
    sets = api.label_sets(b, binn, [to_dev(t) for t in thrs], k)
    torch.cuda.synchronize()
    for i, sg in enumerate(segs):
        assert np.array_equal(one[i].cpu().numpy(), oracle.label(sg, lo, hi, L, thrs[0][i])), (win, k, i)
        for u in range(3):
            assert np.array_equal(sets[u][i].cpu().numpy(), oracle.label(sg, lo, hi, L, thrs[u][i])), (win, k, u, i)


@pytest.mark.parametrize("k", [4, 7, 16])
def test_label_many_thresholds_ragged(ragged, k):
    """k >= 4 thresholds (the DP search's range): labels 0..k bit-exact on
    ragged, unaligned problems, alone and as several sets in one pass."""
    host, base, segs = ragged
    rng = np.random.default_rng(60 + k)
    b = api.Batch(segs)
    for lo, hi, L in [(-1024, 3071, 4096), (-1024, -200, 256), (-5, 7, 13), (3, 1000, 7)]:
        if L - 1 < k:
            continue
        thrs = []
        for u in range(3):
            thr = np.stack([np.sort(rng.choice(L - 1, k, replace=False)) for _ in segs]).astype(np.int32)
            thr[(u + 2) % len(segs)] = -1  # degenerate row
            thrs.append(thr)
        one = api.label(b, api.binning(lo, hi, L), to_dev(thrs[0]), k)
        sets = api.label_sets(b, api.binning(lo, hi, L), [to_dev(t) for t in thrs], k)
        torch.cuda.synchronize()
        for i, sg in enumerate(segs):
            v = sg.cpu().numpy()
            assert np.array_equal(one[i].cpu().numpy(), oracle.label(v, lo, hi, L, thrs[0][i])), (lo, hi, L, k, i)
            for u in range(3):
                want = oracle.label(v, lo, hi, L, thrs[u][i])
                assert np.array_equal(sets[u][i].cpu().numpy(), want), (lo, hi, L, k, u, i)


def test_label_misaligned_output():
    v = to_dev(synth.workload_slice(3).reshape(-1))
    out_buf = torch.empty(v.numel() + 16, dtype=torch.uint8, device=v.device)
    out = out_buf[3:3 + v.numel()]  # output phase differs from the input phase
    thr = to_dev(np.array([[1100]], np.int32))
    api.label(api.Batch([v]), api.binning(-1024, 3071, 4096), thr, 1, outs=[out])
    want = oracle.label(v.cpu().numpy(), -1024, 3071, 4096, [1100])
    assert np.array_equal(out.cpu().numpy(), want)


@pytest.mark.parametrize("nsets", [1, 2, 3, 4])
def test_label_sets_ragged(ragged, nsets):
    """One pass over the voxels, one label map per threshold set, each equal
    to the oracle's labels for that set (ragged, unaligned problems)."""
    host, base, segs = ragged
    rng = np.random.default_rng(40 + nsets)
    b = api.Batch(segs)
    for lo, hi, L in WINDOWS[:4] + WINDOWS[6:7]:
        for k in (1, 2, 3):
            thrs = []
            for u in range(nsets):
                thr = np.stack([np.sort(rng.choice(L - 1, k, replace=False)) for _ in segs]).astype(np.int32)
                thr[(u + 1) % len(segs)] = -1  # a degenerate row in a different problem per set
                thrs.append(thr)
            outs = api.label_sets(b, api.binning(lo, hi, L), [to_dev(t) for t in thrs], k)
            torch.cuda.synchronize()
            for u in range(nsets):
                for i, s in enumerate(segs):
                    want = oracle.label(s.cpu().numpy(), lo, hi, L, thrs[u][i])
                    assert np.array_equal(outs[u][i].cpu().numpy(), want), (lo, hi, L, k, u, i)


def test_label_sets_mixed_output_phases():
    """Sets whose outputs have different alignment phases take the element
    path for the whole problem; labels stay exact."""
    v = to_dev(synth.workload_slice(4).reshape(-1))
    n = v.numel()
    bufs = [torch.empty(n + 16, dtype=torch.uint8, device=v.device) for _ in range(3)]
    outs = [[bufs[0][:n]], [bufs[1][5:5 + n]], [bufs[2][8:8 + n]]]
    thrs = [np.array([[900, 1500]], np.int32), np.array([[100, 2000]], np.int32), np.array([[1, 4000]], np.int32)]
    api.label_sets(api.Batch([v]), api.binning(-1024, 3071, 4096), [to_dev(t) for t in thrs], 2, outs=outs)
    torch.cuda.synchronize()
    for u in range(3):
        want = oracle.label(v.cpu().numpy(), -1024, 3071, 4096, thrs[u][0])
        assert np.array_equal(outs[u][0].cpu().numpy(), want), u


LABEL_TUNES = [dict(label_block=64, label_vecs=1), dict(label_block=256, label_vecs=4),
               dict(label_block=1024, label_vecs=2), dict(label_block=1024, label_vecs=4)]


@pytest.mark.parametrize("tune", LABEL_TUNES, ids=lambda t: f"b{t['label_block']}u{t['label_vecs']}")
def test_label_tuning_invariant(ragged, tune):
    """Every tile shape gives the oracle's labels: ragged unaligned problems,
    slices whose size is not a multiple of the tile (tiles straddle slices),
    and one long problem with a ragged end."""
    host, base, segs = ragged
    rng = np.random.default_rng(77)
    vol = synth.make_volume(synth.rng_for(9, 5), 9, 64)[:, :37, :29].copy()  # 1073-voxel slices
    dv = to_dev(vol)
    long = to_dev(synth.make_volume(synth.rng_for(9, 6), 3, 512).reshape(-1)[:700001].copy())
    cases = [(api.Batch(segs), [s.cpu().numpy() for s in segs]),
             (api.Batch.slices(dv), [vol[z].reshape(-1) for z in range(vol.shape[0])]),
             (api.Batch([long]), [long.cpu().numpy()])]
    lo, hi, L = -1024, 3071, 1024
    for b, hosts in cases:
        for k in (1, 2, 3):
            thrs = [np.stack([np.sort(rng.choice(L - 1, k, replace=False)) for _ in hosts]).astype(np.int32)
                    for _ in range(2)]
            outs = api.label_sets(b, api.binning(lo, hi, L), [to_dev(t) for t in thrs], k, tune=tune)
            one = api.label(b, api.binning(lo, hi, L), to_dev(thrs[0]), k, tune=tune)
            torch.cuda.synchronize()
            for i, h in enumerate(hosts):
                for u in range(2):
                    want = oracle.label(h, lo, hi, L, thrs[u][i])
                    assert np.array_equal(outs[u][i].cpu().numpy(), want), (tune, k, u, i)
                assert np.array_equal(one[i].cpu().numpy(), outs[0][i].cpu().numpy()), (tune, k, i)


def test_determinism_and_batch_invariance():
    vol = synth.make_volume(synth.rng_for(9, 2), 24, 256)
    dv = to_dev(vol)
    binn = api.binning(-1024, -200, 256)
    whole = api.Batch.slices(dv)
    r1 = api.segment_steps(whole, binn, 2, 0.8)
    r2 = api.segment_steps(whole, binn, 2, 0.8)
    torch.cuda.synchronize()
    assert torch.equal(r1[0], r2[0]) and torch.equal(r1[2][0], r2[2][0])
    assert torch.equal(r1[2][1], r2[2][1])
    for a, b in zip(r1[3], r2[3]):
        assert torch.equal(a, b)
    # each slice alone gives the same bits as inside the batch
    for z in (0, 7, 23):
        one = api.segment_steps(api.Batch([dv[z].reshape(-1)]), binn, 2, 0.8)
        assert torch.equal(one[0][0], r1[0][z])
        assert torch.equal(one[2][0][0], r1[2][0][z]) and torch.equal(one[2][1][0], r1[2][1][z])
        assert torch.equal(one[3][0], r1[3][z])
    # the whole path in one call (one workgroup per slice) gives the same bits
    f = api.segment(whole, binn, 2, 0.8, tune={"segment_parts": 1})
    torch.cuda.synchronize()
    assert torch.equal(f[0], r1[0]) and torch.equal(f[1][0], r1[2][0])
    assert torch.equal(f[1][1].view(torch.int64), r1[2][1].view(torch.int64))
    for a, b in zip(f[2][0], r1[3]):
        assert torch.equal(a, b)


@pytest.mark.parametrize("q", [0.5, 1.5])
def test_fused_and_tiled_search_paths_agree(q):
    """The one-workgroup-per-problem kernel and the one-launch-per-phase
    kernels, forced through the tuning, give the same bits; so do batches of
    >= 128 problems (automatic choice: one workgroup per problem) and
    sub-batches of 5 (automatic choice: one launch per phase)."""
    rng = np.random.default_rng(77)
    for k, L in ((1, 300), (2, 300), (2, 1000)):
        H = _random_hists(rng, 140, L, zero_frac=0.15, hi=3000)
        big = _search_all(H, k, q, api.SEARCH_FP32_TIECHECK)
        for path in (1, 2):
            for tb in ((256, 1024) if path == 1 else (512,)):
                forced = _search_all(H, k, q, api.SEARCH_FP32_TIECHECK,
                                     tune=dict(search_path=path, search_block=tb, search_cols=1 + (tb == 1024)))
                for x, y in zip(forced, big):
                    assert np.array_equal(x, y, equal_nan=True), (k, L, path, tb)
        for i0 in (0, 64, 135):
            small = _search_all(H[i0:i0 + 5], k, q, api.SEARCH_FP32_TIECHECK)
            for x, y in zip(small, big):
                assert np.array_equal(x, y[i0:i0 + 5], equal_nan=True), (k, L, i0)
        for i in range(0, 140, 23):
            check_choice(H[i], k, q, big[0][i], big[1][i], big[2][i])


@pytest.mark.parametrize("q", [0.8, 1.5])
def test_search_k3_column_chunks(q):
    """k = 3 rows longer than one 1024-column chunk (L = 1100), two problems
    in one batch, against the oracle (prefix mode)."""
    rng = np.random.default_rng(91)
    H = _random_hists(rng, 2, 1100, zero_frac=0.25, hi=4000)
    H[0, 500:540] = 0  # a run of empty bins
    thr, obj, st = _search_all(H, 3, q, api.SEARCH_FP32_TIECHECK)
    for i in range(2):
        check_choice(H[i], 3, q, thr[i], obj[i], st[i])


QBATCH = (0.5, 1.5, 0.8, 2.0, 1.0, 1.2, 0.3, 3.0)  # both signs of 1 - q and the Shannon limit; TS_MAX_Q values


def test_prefix_batched_q_equals_single_calls():
    rng = np.random.default_rng(71)
    H = _random_hists(rng, 9, 777, zero_frac=0.5, hi=2000)
    H[3] = 0  # empty problem
    hd = to_dev(H.view(np.int32))
    P, Q = api.prefix(hd, QBATCH)
    assert tuple(Q.shape) == (len(QBATCH), 9, 777)
    for j, q in enumerate(QBATCH):
        P1, Q1 = api.prefix(hd, q)
        assert torch.equal(P, P1)
        assert torch.equal(Q[j], Q1), q


@pytest.mark.parametrize("mode", MODES, ids=["fp32tie", "fp64", "plain"])
@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("path", [0, 1, 2], ids=["auto", "fused", "tiled"])
def test_search_batched_q_equals_single_calls(mode, k, path):
    """One launch over nq x nseg problems gives, bit for bit, what nq calls
    with one q give; the results also match the oracle."""
    if path and mode != api.SEARCH_FP32_TIECHECK:
        pytest.skip("paths only differ in the FP32 mode")
    rng = np.random.default_rng(500 + 10 * k + mode + path)
    L = {1: 300, 2: 130, 3: 40}[k] if mode == api.SEARCH_PLAIN else {1: 1000, 2: 257, 3: 70}[k]
    n = 3 if mode == api.SEARCH_PLAIN else 7
    H = _random_hists(rng, n, L, zero_frac=0.4)
    H[1] = 0
    H[1, 5] = 3  # one occupied bin: degenerate
    qs = QBATCH[:3] if mode == api.SEARCH_PLAIN else QBATCH
    tune = {"search_path": path} if path else None
    hd = to_dev(H.view(np.int32))
    P, Q = api.prefix(hd, qs)
    thr, obj, st = api.threshold_search(P, Q, k, qs, mode, tune=tune)
    torch.cuda.synchronize()
    assert tuple(thr.shape) == (len(qs), n, k)
    for j, q in enumerate(qs):
        P1, Q1 = api.prefix(hd, q)
        t1, o1, s1 = api.threshold_search(P1, Q1, k, q, mode, tune=tune)
        torch.cuda.synchronize()
        assert torch.equal(thr[j], t1), (q, thr[j], t1)
        assert torch.equal(st[j], s1), q
        o = obj[j].cpu().numpy()
        assert np.array_equal(o, o1.cpu().numpy(), equal_nan=True), q
        if mode == api.SEARCH_FP32_TIECHECK:
            sj = st[j].cpu().numpy()
            om = oracle.MODE_KAPUR if q == 1.0 else oracle.MODE_PREFIX
            for i in range(n):
                check_choice(H[i], k, q, thr[j, i].cpu().numpy(), o[i], int(sj[i]), mode=om)


def test_v_log_f32_error_within_the_search_bound():
    """The FP32 logarithm of the search keys is within LOG2_ERR_UNITS = 4
    units of 2^-24 * max(1, |log2 x|) of log2(x) (FP64) over normal inputs
    from 2^-126 to 2^64 (class sums of the search live in this range; the
    error bound falls back to a full FP64 check below 1e-36)."""
    rng = np.random.default_rng(2024)
    e = rng.integers(-126, 64, 4_000_000)
    m = rng.random(4_000_000)
    x = np.ldexp(1.0 + m, e).astype(np.float32)
    x = np.concatenate([x, np.float32([1.0, 2.0, 0.5, 1.0000001, 0.99999994]),
                        np.nextafter(np.float32(1.0), np.float32(0.0), dtype=np.float32)[None],
                        np.float32(np.linspace(0.5, 2.0, 200001))])
    y = api.log2_f32(to_dev(x)).cpu().numpy().astype(np.float64)
    exact = np.log2(x.astype(np.float64))
    units = np.abs(y - exact) / (2.0 ** -24 * np.maximum(1.0, np.abs(exact)))
    worst = float(units.max())
    say(f"v_log_f32: worst error {worst:.3f} units of 2^-24*max(1,|log2 x|)")
    assert worst <= 4.0, (worst, x[int(units.argmax())])
