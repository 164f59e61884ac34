"""ts_segment (the whole path in one call) against the four separate calls
(ts_histogram, ts_prefix, ts_threshold_search, ts_label_sets) on the same
inputs: histograms, thresholds, FP64 objectives (bit patterns), statuses and
labels identical bit for bit, for one workgroup per problem (everything in
one launch) and several (last workgroup searches, then the label pass), the
separate-pass fallback (k = 3, FP64 mode), ragged and misaligned problems,
empty problems, and one workspace of any contents reused over calls; a sample
also against the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import check_choice, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2012_10684_amd import api, synth  # noqa: E402


def _steps(batch, binn, k, qs, mode=api.SEARCH_FP32_TIECHECK):
    h = api.histogram(batch, binn)
    P, Q = api.prefix(h, qs)
    thr, obj, st = api.threshold_search(P, Q, k, qs, mode)
    labs = api.label_sets(batch, binn, [thr[j] for j in range(len(qs))], k)
    return h, (thr, obj, st), labs


def _same(a, b, where):
    (ha, (ta, oa, sa), la), (hb, (tb, ob, sb), lb) = a, b
    assert torch.equal(ha, hb), where
    assert torch.equal(ta, tb), (where, ta, tb)
    assert torch.equal(oa.view(torch.int64), ob.view(torch.int64)), (where, oa, ob)
    assert torch.equal(sa, sb), where
    if la is not None and lb is not None:
        for j in range(len(la)):
            for i in range(len(la[j])):
                assert torch.equal(la[j][i], lb[j][i]), (where, j, i)


@pytest.fixture(scope="module")
def slices():
    return synth.workload_volume300(0)[:40].copy()  # 40 slices of 512 x 512


@pytest.mark.parametrize("parts", [0, 1, 2, 5])
def test_per_slice_k2_three_q(slices, parts):
    binn = api.binning(-1024, -200, 256)
    qs = [0.5, 0.8, 1.5]
    dv = to_dev(slices)
    b = api.Batch.slices(dv)
    tune = {"segment_parts": parts} if parts else None
    say(f"segment per slice k=2 L=256 nq=3 parts={parts or 'default'}")
    got = api.segment(b, binn, 2, qs, tune=tune)
    want = _steps(b, binn, 2, qs)
    torch.cuda.synchronize()
    _same(got, want, parts)
    H = got[0].cpu().numpy().view(np.uint32)
    thr, obj, st = (x.cpu().numpy() for x in got[1])
    for z in (0, 17, 39):
        assert np.array_equal(H[z], oracle.histogram(slices[z], -1024, -200, 256))
        for j, q in enumerate(qs):
            check_choice(H[z], 2, q, thr[j][z], obj[j][z], st[j][z])


@pytest.mark.parametrize("parts", [0, 1, 16, 64])
def test_one_slice_4096_bins_k1(parts):
    img = synth.workload_slice(0)
    binn = api.binning(-1024, 3071, 4096)
    b = api.Batch([to_dev(img).reshape(-1)])
    tune = {"segment_parts": parts} if parts else None
    say(f"segment one slice k=1 L=4096 parts={parts or 'default'}")
    got = api.segment(b, binn, 1, 0.8, tune=tune)
    want = _steps(b, binn, 1, [0.8])
    torch.cuda.synchronize()
    want = (want[0], tuple(x[0] for x in want[1]), want[2])
    _same(got, want, parts)
    h = oracle.histogram(img, -1024, 3071, 4096)
    assert np.array_equal(got[0].cpu().numpy().view(np.uint32)[0], h)
    check_choice(h, 1, 0.8, got[1][0].cpu().numpy()[0], got[1][1].item(), got[1][2].item())
    want_l = oracle.label(img.reshape(-1), -1024, 3071, 4096, got[1][0].cpu().numpy()[0])
    assert np.array_equal(got[2][0][0].cpu().numpy(), want_l)


def _ragged():
    """Problems of sizes 0, 1, 7, 8, 9, 1000, 65536 + 3 and a 512 x 512 slice,
    at odd element offsets of one buffer (2-byte aligned pointers)."""
    rng = np.random.default_rng(7)
    sizes = [0, 1, 7, 8, 9, 1000, 65539, 262144, 0, 5]
    buf = rng.normal(-300, 700, sum(sizes) + 64).clip(-1024, 3071).astype(np.int16)
    buf[::97] = -32768
    buf[5::101] = 32767
    return buf, sizes


@pytest.mark.parametrize("k,L,lo,hi,parts", [(1, 1000, -1024, 3071, 0), (2, 256, -1024, -200, 0),
                                             (2, 256, -1024, -200, 3), (1, 4096, -1024, 3071, 2),
                                             (2, 1024, -5, 7, 1), (1, 13, -5, 7, 4)])
def test_ragged_misaligned(k, L, lo, hi, parts):
    buf, sizes = _ragged()
    dbuf = to_dev(buf)
    segs, o = [], 3  # odd start: 2-byte aligned only
    for n in sizes:
        segs.append(dbuf[o:o + n])
        o += n
    b = api.Batch(segs)
    binn = api.binning(lo, hi, L)
    qs = [0.8, 1.5]
    tune = {"segment_parts": parts} if parts else None
    say(f"segment ragged k={k} L={L} [{lo},{hi}] parts={parts or 'default'}")
    got = api.segment(b, binn, k, qs, tune=tune)
    want = _steps(b, binn, k, qs)
    torch.cuda.synchronize()
    _same(got, want, (k, L, parts))
    st = got[1][2].cpu().numpy()
    assert st[0][0] == api.PROBLEM_EMPTY and st[0][8] == api.PROBLEM_EMPTY


def test_fallback_k3_and_fp64(slices):
    binn = api.binning(-1024, 3071, 512)
    dv = to_dev(slices[:4])
    b = api.Batch([dv.reshape(-1)])  # one problem of 4 slices
    say("segment fallback k=3 (separate passes)")
    got = api.segment(b, binn, 3, 0.8)
    want = _steps(b, binn, 3, [0.8])
    torch.cuda.synchronize()
    _same(got, (want[0], tuple(x[0] for x in want[1]), want[2]), "k3")
    say("segment fallback FP64 mode")
    b2 = api.Batch.slices(dv)
    got = api.segment(b2, api.binning(-1024, -200, 256), 2, 0.8, mode=api.SEARCH_FP64)
    want = _steps(b2, api.binning(-1024, -200, 256), 2, [0.8], mode=api.SEARCH_FP64)
    torch.cuda.synchronize()
    _same(got, (want[0], tuple(x[0] for x in want[1]), want[2]), "fp64")


def test_workspace_contents_ignored(slices):
    """Calls of different sizes share one workspace whose contents are
    garbage or left by other calls: each call tags its tickets, so the last
    part of every problem is found whatever the words held."""
    binn = api.binning(-1024, -200, 256)
    dv = to_dev(slices)
    need = api.segment_workspace_bytes(40, 256, 2, 1)
    ws = torch.full((need,), 0xFF, dtype=torch.uint8, device=dv.device)
    g = torch.Generator(device=dv.device)
    g.manual_seed(3)
    for n, parts, junk in [(40, 4, False), (7, 9, False), (40, 2, True), (1, 64, False), (13, 1, True),
                           (40, 4, False), (40, 4, False)]:
        say(f"segment reuse: {n} slices, parts {parts}, junk {junk}")
        if junk:
            ws.random_(0, 256, generator=g)
        b = api.Batch.slices(dv[:n])
        got = api.segment(b, binn, 2, 0.8, ws=ws, tune={"segment_parts": parts})
        want = _steps(b, binn, 2, [0.8])
        torch.cuda.synchronize()
        _same(got, (want[0], tuple(x[0] for x in want[1]), want[2]), (n, parts))


def test_without_labels(slices):
    binn = api.binning(-1024, -200, 256)
    b = api.Batch.slices(to_dev(slices[:9]))
    got = api.segment(b, binn, 2, [0.5, 1.5], labels=False)
    want = _steps(b, binn, 2, [0.5, 1.5])
    torch.cuda.synchronize()
    assert got[2] is None
    _same(got, want, "no labels")


def _one_problem_inputs():
    """One problem per entry: a workload slice, a constant image, tiny and
    ragged sizes at odd element offsets (2-byte aligned), four slices."""
    rng = np.random.default_rng(11)
    img = synth.workload_slice(0).reshape(-1)
    buf = rng.normal(-300, 700, 70000).clip(-1024, 3071).astype(np.int16)
    buf[::97] = -32768
    buf[5::101] = 32767
    four = synth.workload_volume300(0)[:4].reshape(-1)
    return [("slice", img), ("constant", np.full(5000, -600, np.int16)), ("one", buf[3:4]),
            ("nine", buf[3:12]), ("ragged", buf[3:65542]), ("four slices", four)]


@pytest.mark.parametrize("L,lo,hi", [(4096, -1024, 3071), (1000, -1024, 3071), (256, -1024, -200), (13, -5, 7),
                                     (2, -1024, 3071)])
@pytest.mark.parametrize("q", [0.5, 0.8, 1.0, 3.0])
def test_one_problem_path(L, lo, hi, q):
    """ts_segment for one problem, k = 1, one q (the cooperative path that
    spreads the prefix sums and the search over many workgroups) against the
    separate calls bit for bit, labels included; with and without labels."""
    binn = api.binning(lo, hi, L)
    for name, v in _one_problem_inputs():
        dv = to_dev(np.ascontiguousarray(v))
        b = api.Batch([dv])
        say(f"one-problem path L={L} q={q} {name} ({v.size} voxels)")
        got = api.segment(b, binn, 1, q)
        want = _steps(b, binn, 1, [q])
        torch.cuda.synchronize()
        want = (want[0], tuple(x[0] for x in want[1]), want[2])
        _same(got, want, (L, q, name))
        nolab = api.segment(b, binn, 1, q, labels=False)
        torch.cuda.synchronize()
        assert nolab[2] is None
        _same((nolab[0], nolab[1], None), (want[0], want[1], None), (L, q, name, "no labels"))
        if name == "constant":
            assert got[1][2].item() == api.PROBLEM_DEGENERATE


def test_one_problem_path_oracle_and_reuse():
    """The one-problem path against the oracle, and one workspace of any
    contents reused over calls of different sizes (the barrier word carries
    each call's tag)."""
    img = synth.workload_slice(1)
    binn = api.binning(-1024, 3071, 4096)
    dv = to_dev(img.reshape(-1))
    need = api.segment_workspace_bytes(1, 4096, 1, 1)
    ws = torch.full((need,), 0xFF, dtype=torch.uint8, device=dv.device)
    h = oracle.histogram(img, -1024, 3071, 4096)
    for n, junk in [(img.size, False), (1000, True), (img.size, True), (77777, False), (img.size, False)]:
        say(f"one-problem path reuse: {n} voxels, junk {junk}")
        if junk:
            ws.random_(0, 256)
        b = api.Batch([dv[:n]])
        got = api.segment(b, binn, 1, 0.8, ws=ws)
        want = _steps(b, binn, 1, [0.8])
        torch.cuda.synchronize()
        _same(got, (want[0], tuple(x[0] for x in want[1]), want[2]), (n, junk))
    got = api.segment(api.Batch([dv]), binn, 1, 0.8, ws=ws)
    torch.cuda.synchronize()
    assert np.array_equal(got[0].cpu().numpy().view(np.uint32)[0], h)
    check_choice(h, 1, 0.8, got[1][0].cpu().numpy()[0], got[1][1].item(), got[1][2].item())
