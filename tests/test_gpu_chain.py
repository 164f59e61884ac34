"""The paper's own segmentation step, composed on the GPU and checked stage by
stage against the oracle: each gray-level image is opened by the disk of
radius 10 (Morphology section) and the residue (original - opened) is
thresholded by the two-dimensional Tsallis form (Tsallis-entropy section):
the 2D histogram of (gray level, 3x3 average gray level) of the residue, the
arg max pair (t, s) over quadrants 1 and 3, and the residue labelled by t
alone (only t thresholds the image).  Residue levels are their own bins
(identity binning {0, L-1, L}).  Histograms and labels bit-exact; the pair
identical unless the oracle's best two are within 1e-6 relative; objective
within 1e-5 relative."""
import numpy as np
import pytest

import oracle
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2012_10684_amd import api, synth  # noqa: E402

LO, HI, L, R = -1024, -200, 256, 10
QS = [0.5, 0.8, 1.5]


@pytest.fixture(scope="module")
def chain_inputs():
    vol = synth.workload_volume300(0)[::100].copy()  # 3 slices of 512 x 512
    want = []
    for img in vol:
        _, res = oracle.opening(oracle.gray(img, LO, HI, L), R)
        r16 = res.astype(np.int16)
        want.append((r16, oracle.histogram2d(r16, 0, L - 1, L)))
    return vol, want


def _check_pair(h2, q, t, s, obj, status):
    r = oracle.search2d(h2, q, oracle.MODE_PREFIX)
    assert r.status == oracle.OK and status == 0, (r, status)
    if [t, s] != r.thr.tolist():
        s_gpu = oracle.objective2d(h2, t, s, q, oracle.MODE_PREFIX)
        assert s_gpu >= r.obj - 1e-6 * abs(r.obj), ([t, s], r)
    assert abs(obj - r.obj) <= 1e-5 * abs(r.obj) + 1e-12, (obj, r)
    return r


def test_paper_segmentation_chain(chain_inputs):
    vol, want = chain_inputs
    n, H, W = vol.shape
    say(f"chain: {n} images {H}x{W}, radius {R}, q {QS}")
    dv = to_dev(vol)
    _, _, r16 = api.open2d(api.Batch.slices(dv), H, W, api.binning(LO, HI, L), R, want=("residue16",))
    ident = api.binning(0, L - 1, L)
    b = api.Batch.slices(r16)
    h2 = api.histogram2d(b, H, W, ident)
    thr, obj, st = api.threshold_search2d(h2, QS)  # [nq, 2, n]
    labels = api.label_sets(b, ident, [thr[j, 0] for j in range(len(QS))], 1)
    torch.cuda.synchronize()
    R16 = r16.cpu().numpy()
    Hg = h2.cpu().numpy().view(np.uint32)
    thr, obj, st = thr.cpu().numpy(), obj.cpu().numpy(), st.cpu().numpy()
    for i, (r16w, h2w) in enumerate(want):
        assert np.array_equal(R16[i], r16w), i
        assert np.array_equal(Hg[i], h2w), i
        for j, q in enumerate(QS):
            t, s = int(thr[j, 0, i]), int(thr[j, 1, i])
            _check_pair(h2w, q, t, s, obj[j, i], st[j, i])
            lab = labels[j][i].cpu().numpy()
            assert np.array_equal(lab, oracle.label(r16w.reshape(-1), 0, L - 1, L, np.array([t]))), (i, q)
    say(f"chain pairs (t, s): {[[(int(thr[j, 0, i]), int(thr[j, 1, i])) for i in range(n)] for j in range(len(QS))]}")


def test_batch_segment_2d_with_opening_equals_the_stages(chain_inputs):
    """api.batch_segment(method="2d", open_radius=10) gives the same 2D
    histograms, pairs, objectives and labels as the stages called one by
    one (it only marshals them)."""
    vol, want = chain_inputs
    n, H, W = vol.shape
    dv = to_dev(vol)
    seg = api.batch_segment([dv[:2], dv[2:]], api.binning(LO, HI, L), 1, QS, per="slice", method="2d",
                            open_radius=R)
    torch.cuda.synchronize()
    Hg = seg.hist.cpu().numpy().view(np.uint32)
    thr = seg.thr.cpu().numpy()  # [nq, n, 2]
    for i, (r16w, h2w) in enumerate(want):
        assert np.array_equal(Hg[i], h2w), i
        for j, q in enumerate(QS):
            t, s = int(thr[j, i, 0]), int(thr[j, i, 1])
            _check_pair(h2w, q, t, s, seg.obj[j, i].item(), seg.status[j, i].item())
            v, z = (0, i) if i < 2 else (1, i - 2)
            lab = seg.labels[j][v][z].cpu().numpy().reshape(-1)
            assert np.array_equal(lab, oracle.label(r16w.reshape(-1), 0, L - 1, L, np.array([t]))), (i, q)
