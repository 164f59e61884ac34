"""GPU parity of the two-dimensional method (2D histogram of gray level and
3x3 average gray level, arg max over threshold pairs) against the oracle:
2D histograms bit-exact, pairs identical unless the oracle's best two
objectives are within 1e-6 relative (then the GPU pair's oracle objective
must be within 1e-6 of the best), objectives within 1e-5 relative."""
import numpy as np
import pytest

import oracle
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2012_10684_amd import api, synth  # noqa: E402

WINDOWS = [(-1024, 3071, 256), (-1024, -200, 256), (-1024, 3071, 64), (-5, 7, 13), (100, 100, 4), (-32768, 32767, 200)]


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def check_pair(h2, q, thr, obj, status):
    mode = oracle.MODE_KAPUR if q == 1.0 else (oracle.MODE_DIRECT if h2.shape[0] <= 24 else oracle.MODE_PREFIX)
    r = oracle.search2d(h2, q, mode)
    if r.status != oracle.OK:
        assert status == r.status and list(thr) == [-1, -1] and np.isnan(obj), (status, r)
        return
    assert status == 0, (status, r)
    if list(thr) != r.thr.tolist():
        s_gpu = oracle.objective2d(h2, int(thr[0]), int(thr[1]), q, mode)
        assert s_gpu >= r.obj - 1e-6 * abs(r.obj), (list(thr), r)
    assert abs(obj - r.obj) <= 1e-5 * abs(r.obj) + 1e-12, (obj, r)


@pytest.mark.parametrize("win", WINDOWS, ids=lambda w: f"{w[0]}_{w[1]}_{w[2]}")
def test_histogram2d_matches_oracle(win):
    lo, hi, L = win
    rng = np.random.default_rng(abs(lo) + L)
    for H, W in [(1, 1), (1, 7), (5, 1), (3, 3), (37, 29), (64, 61), (130, 512)]:
        n = 3
        if L >= 64 and min(H, W) >= 24:  # CT-like images (the tube generator needs room)
            imgs = synth.make_volume(synth.rng_for(9, H * W % 97), n, max(H, W))[:, :H, :W].copy()
        elif L >= 64:
            imgs = rng.normal(-300, 700, (n, H, W)).clip(-1024, 3071).astype(np.int16)
        else:
            imgs = rng.integers(lo - 20, hi + 20, (n, H, W)).astype(np.int16)
        imgs[0, 0, 0] = -32768
        imgs[-1, -1, -1] = 32767
        dv = to_dev(imgs)
        h = u32(api.histogram2d(api.Batch.slices(dv), H, W, api.binning(lo, hi, L)))
        torch.cuda.synchronize()
        for i in range(n):
            want = oracle.histogram2d(imgs[i], lo, hi, L)
            assert np.array_equal(h[i], want), (win, H, W, i)


def test_histogram2d_noisy_images_use_the_global_path():
    """Uniform noise puts most (f, g) pairs far from the diagonal."""
    rng = np.random.default_rng(3)
    imgs = rng.integers(-1024, 3072, (2, 200, 300)).astype(np.int16)
    h = u32(api.histogram2d(api.Batch.slices(to_dev(imgs)), 200, 300, api.binning(-1024, 3071, 256)))
    for i in range(2):
        assert np.array_equal(h[i], oracle.histogram2d(imgs[i], -1024, 3071, 256))


def _rand_h2(rng, L, zero_frac=0.5, hi=30):
    h = rng.integers(0, hi, (L, L)).astype(np.uint32)
    h[rng.random((L, L)) < zero_frac] = 0
    return h


@pytest.mark.parametrize("q", [0.3, 0.8, 1.0, 1.5, 3.0])
def test_search2d_small_random(q):
    rng = np.random.default_rng(int(q * 100) + 5)
    for L in (2, 3, 7, 16, 33, 100):
        H2 = np.stack([_rand_h2(rng, L) for _ in range(4)])
        thr, obj, st = api.threshold_search2d(to_dev(H2.view(np.int32)), q)
        thr, obj, st = thr.cpu().numpy(), obj.cpu().numpy(), st.cpu().numpy()
        for i in range(len(H2)):
            check_pair(H2[i], q, thr[:, i], obj[i], st[i])


def test_search2d_edge_cases():
    L = 8
    H2 = np.zeros((4, L, L), np.uint32)
    H2[1, 3, 4] = 10  # one cell: degenerate
    H2[2, 3, 4] = 10
    H2[2, 6, 6] = 4  # all valid pairs tie at S = 0: the first, (3, 4)
    H2[3] = 5  # uniform: (L/2 - 1, L/2 - 1)
    thr, obj, st = api.threshold_search2d(to_dev(H2.view(np.int32)), 0.8)
    thr, st = thr.cpu().numpy().T, st.cpu().numpy()
    assert st.tolist() == [api.PROBLEM_EMPTY, api.PROBLEM_DEGENERATE, 0, 0]
    assert thr[0].tolist() == [-1, -1] and thr[1].tolist() == [-1, -1]
    assert thr[2].tolist() == [3, 4] and obj[2].item() == 0.0
    assert thr[3].tolist() == [L // 2 - 1, L // 2 - 1]


def test_search2d_batched_q_equals_single_calls():
    rng = np.random.default_rng(11)
    H2 = np.stack([_rand_h2(rng, 48, zero_frac=0.6) for _ in range(5)])
    hd = to_dev(H2.view(np.int32))
    qs = (0.5, 1.5, 1.0, 0.8)
    thr, obj, st = api.threshold_search2d(hd, qs)
    for j, q in enumerate(qs):
        t1, o1, s1 = api.threshold_search2d(hd, q)
        assert torch.equal(thr[j], t1) and torch.equal(st[j], s1)
        assert np.array_equal(obj[j].cpu().numpy(), o1.cpu().numpy(), equal_nan=True)


@pytest.mark.parametrize("q", [0.8, 1.5])
def test_search2d_workload_slices(q):
    """Slices of the 300-slice workload, 256 gray levels over [-1024, -200]:
    2D histograms, pairs against the oracle, and labels from t."""
    vol = synth.workload_volume300(0)[::75]
    dv = to_dev(vol)
    b = api.Batch.slices(dv)
    binn = api.binning(-1024, -200, 256)
    h2 = api.histogram2d(b, 512, 512, binn)
    thr, obj, st = api.threshold_search2d(h2, q)
    labels = api.label(b, binn, thr[0], 1)  # row 0 (t) is the k = 1 threshold array
    torch.cuda.synchronize()
    H2, thr_h, obj_h, st_h = u32(h2), thr.cpu().numpy().T, obj.cpu().numpy(), st.cpu().numpy()
    for z in range(vol.shape[0]):
        want = oracle.histogram2d(vol[z], -1024, -200, 256)
        assert np.array_equal(H2[z], want), z
        check_pair(want, q, thr_h[z], obj_h[z], st_h[z])
        lab = oracle.label(vol[z].reshape(-1), -1024, -200, 256, thr_h[z][:1])
        assert np.array_equal(labels[z].cpu().numpy(), lab), z
    say(f"2-D pairs at q={q}: {thr_h.tolist()}")


@pytest.mark.parametrize("L", [129, 254, 255, 256])
def test_search2d_wide_histograms(L):
    """Widths up to the 256-level maximum, including ones that leave a lane
    with fewer than four columns."""
    rng = np.random.default_rng(L)
    H2 = np.stack([_rand_h2(rng, L, zero_frac=0.7, hi=200) for _ in range(2)])
    for q in (0.6, 1.4):
        thr, obj, st = api.threshold_search2d(to_dev(H2.view(np.int32)), q)
        thr, obj, st = thr.cpu().numpy(), obj.cpu().numpy(), st.cpu().numpy()
        for i in range(len(H2)):
            check_pair(H2[i], q, thr[:, i], obj[i], st[i])


def test_search2d_empty_rows_and_columns():
    """Runs of empty gray levels (rows) and empty average levels (columns)
    make whole blocks of pairs tie exactly; the first pair must win, as in
    the oracle."""
    rng = np.random.default_rng(21)
    L = 64
    cases = []
    for k in range(6):
        h = _rand_h2(rng, L, zero_frac=0.4)
        rows = rng.choice(L, size=L // 2, replace=False)
        cols = rng.choice(L, size=L // 3, replace=False)
        h[rows, :] = 0
        h[:, cols] = 0
        cases.append(h)
    banded = np.zeros((L, L), np.uint32)  # two blobs separated by empty rows and columns
    banded[2:10, 3:12] = rng.integers(1, 50, (8, 9))
    banded[40:50, 45:60] = rng.integers(1, 50, (10, 15))
    cases.append(banded)
    H2 = np.stack(cases)
    for q in (0.5, 1.0, 2.0):
        thr, obj, st = api.threshold_search2d(to_dev(H2.view(np.int32)), q)
        thr, obj, st = thr.cpu().numpy(), obj.cpu().numpy(), st.cpu().numpy()
        for i in range(len(H2)):
            check_pair(H2[i], q, thr[:, i], obj[i], st[i])
        r = oracle.search2d(banded, q, oracle.MODE_KAPUR if q == 1.0 else oracle.MODE_PREFIX)
        assert thr[:, -1].tolist() == r.thr.tolist(), (q, thr[:, -1], r)


def test_search2d_counts_beyond_32_bits():
    """Histograms whose total exceeds 2^32 (and one row that does alone)."""
    rng = np.random.default_rng(7)
    L = 20
    a = rng.integers(0, 1 << 28, (L, L)).astype(np.uint32)
    a[rng.random((L, L)) < 0.3] = 0
    b = _rand_h2(rng, L, zero_frac=0.3)
    b[5, :] = 0xF0000000  # this row alone sums to 20 * 0xF0000000
    H2 = np.stack([a, b])
    assert int(a.astype(np.int64).sum()) > 1 << 32
    for q in (0.7, 1.0, 1.6):
        thr, obj, st = api.threshold_search2d(to_dev(H2.view(np.int32)), q)
        thr, obj, st = thr.cpu().numpy(), obj.cpu().numpy(), st.cpu().numpy()
        for i in range(len(H2)):
            check_pair(H2[i], q, thr[:, i], obj[i], st[i])
