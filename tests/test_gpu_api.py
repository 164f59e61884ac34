"""GPU checks of the Python convenience batch_segment (marshalling over the
C ABI): volumes of uneven depth per slice and per volume, several q in one
pass, k = 4 through the DP search, and the opening first; every problem's
histogram, thresholds and labels against the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import check_choice, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2012_10684_amd import api  # noqa: E402


def _vols(rng, shapes):
    out = []
    for z, h, w in shapes:
        v = rng.normal(-500, 450, (z, h, w))
        v[:, : h // 3] = rng.normal(-950, 40, (z, h // 3, w))  # an air band
        out.append(v.clip(-1024, 3071).astype(np.int16))
    return out


def test_batch_segment_per_slice_several_q():
    rng = np.random.default_rng(5)
    vols = _vols(rng, [(3, 40, 56), (5, 33, 47)])
    lo, hi, L, k, qs = -1024, -200, 128, 2, (0.5, 1.5)
    res = api.batch_segment([to_dev(v) for v in vols], api.binning(lo, hi, L), k, qs, per="slice")
    torch.cuda.synchronize()
    H = res.hist.cpu().numpy().view(np.uint32)
    thr, obj, st = res.thr.cpu().numpy(), res.obj.cpu().numpy(), res.status.cpu().numpy()
    i = 0
    for vi, v in enumerate(vols):
        for z in range(v.shape[0]):
            h = oracle.histogram(v[z].reshape(-1), lo, hi, L)
            assert np.array_equal(H[i], h), (vi, z)
            for j, q in enumerate(qs):
                check_choice(h, k, q, thr[j, i], obj[j, i], st[j, i])
                want = oracle.label(v[z].reshape(-1), lo, hi, L, thr[j, i]).reshape(v.shape[1:])
                assert np.array_equal(res.labels[j][vi][z].cpu().numpy(), want), (vi, z, q)
            i += 1


def test_batch_segment_per_volume_k4_by_dp():
    rng = np.random.default_rng(6)
    vols = _vols(rng, [(4, 30, 30), (2, 50, 20)])
    lo, hi, L, k, q = -1024, 3071, 48, 4, 0.8
    res = api.batch_segment([to_dev(v) for v in vols], api.binning(lo, hi, L), k, q, per="volume")
    torch.cuda.synchronize()
    thr, obj, st = res.thr.cpu().numpy(), res.obj.cpu().numpy(), res.status.cpu().numpy()
    for vi, v in enumerate(vols):
        h = oracle.histogram(v.reshape(-1), lo, hi, L)
        check_choice(h, k, q, thr[0, vi], obj[0, vi], st[0, vi])
        want = oracle.label(v.reshape(-1), lo, hi, L, thr[0, vi]).reshape(v.shape)
        assert np.array_equal(res.labels[0][vi].cpu().numpy(), want), vi


def test_batch_segment_after_the_opening():
    rng = np.random.default_rng(7)
    vols = _vols(rng, [(2, 64, 70), (3, 45, 90)])
    lo, hi, L, k, q, r = -1024, -200, 256, 1, 0.8, 5
    res = api.batch_segment([to_dev(v) for v in vols], api.binning(lo, hi, L), k, q, per="slice", open_radius=r)
    torch.cuda.synchronize()
    thr, obj, st = res.thr.cpu().numpy(), res.obj.cpu().numpy(), res.status.cpu().numpy()
    i = 0
    for vi, v in enumerate(vols):
        for z in range(v.shape[0]):
            _, rr = oracle.opening(oracle.gray(v[z], lo, hi, L), r)
            rr16 = rr.astype(np.int16).reshape(-1)
            h = oracle.histogram(rr16, 0, L - 1, L)
            check_choice(h, k, q, thr[0, i], obj[0, i], st[0, i])
            want = oracle.label(rr16, 0, L - 1, L, thr[0, i]).reshape(v.shape[1:])
            assert np.array_equal(res.labels[0][vi][z].cpu().numpy(), want), (vi, z)
            i += 1


def test_batch_segment_on_a_side_stream():
    """Given a stream, every kernel and every tensor the call makes is on
    that stream: after synchronising it alone the results equal those of a
    call on the current stream, bit for bit."""
    rng = np.random.default_rng(9)
    vols = [to_dev(v) for v in _vols(rng, [(4, 64, 72), (2, 31, 45)])]
    binn = api.binning(-1024, -200, 256)
    ref = api.batch_segment(vols, binn, 2, (0.8, 1.5), per="slice")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    got = api.batch_segment(vols, binn, 2, (0.8, 1.5), per="slice", stream=s)
    s.synchronize()
    assert torch.equal(got.hist, ref.hist) and torch.equal(got.thr, ref.thr) and torch.equal(got.status, ref.status)
    assert torch.equal(got.obj.view(torch.int64), ref.obj.view(torch.int64))
    for j in range(2):
        for vi in range(len(vols)):
            assert torch.equal(got.labels[j][vi], ref.labels[j][vi]), (j, vi)
