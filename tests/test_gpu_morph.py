"""GPU parity of the morphology step (ts_open2d) against the oracle: the
opened image and the residue gray - opened bit-exact, for radii 0..32,
images smaller than a tile or than the disk, sizes that leave ragged tiles,
images wider than a tile,
narrow and wide windows, CT-like slices of the workload, and each output
requested alone."""
import numpy as np
import pytest

import oracle
from gpu_util import check_choice, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2012_10684_amd import api, synth  # noqa: E402


def _check(imgs, lo, hi, L, r, want=("opened", "residue")):
    n, H, W = imgs.shape
    dv = to_dev(imgs)
    o, res, r16 = api.open2d(api.Batch.slices(dv), H, W, api.binning(lo, hi, L), r, want=want)
    torch.cuda.synchronize()
    for i in range(n):
        g = oracle.gray(imgs[i], lo, hi, L)
        oo, rr = oracle.opening(g, r)
        if o is not None:
            assert np.array_equal(o[i].cpu().numpy().astype(np.int32), oo), (H, W, r, i)
        if res is not None:
            assert np.array_equal(res[i].cpu().numpy().astype(np.int32), rr), (H, W, r, i)
        if r16 is not None:
            assert np.array_equal(r16[i].cpu().numpy().astype(np.int32), rr), (H, W, r, i)


@pytest.mark.parametrize("r", [0, 1, 2, 3, 5, 10, 17, 31, 32])
def test_open2d_random_images(r):
    rng = np.random.default_rng(r + 1)
    for H, W in [(1, 1), (3, 200), (64, 64), (70, 129), (130, 65)]:
        imgs = rng.integers(-1100, 400, (2, H, W)).astype(np.int16)
        _check(imgs, -1024, 3071, 256, r)


@pytest.mark.parametrize("r", range(api.MORPH_MAX_RADIUS + 1))
def test_open2d_every_radius(r):
    """Every radius the entry point takes (each has a kernel of its own, in
    one of several sources): images of one tile with ragged rows, and a wide
    image of several tiles with halo columns."""
    rng = np.random.default_rng(900 + r)
    for n, H, W in [(2, 45, 70), (1, 11, 700)]:
        imgs = rng.integers(-1100, 400, (n, H, W)).astype(np.int16)
        _check(imgs, -1024, 3071, 256, r)


@pytest.mark.parametrize("r", [1, 4, 10, 32])
def test_open2d_wide_images(r):
    """Images wider than one tile (512 columns): tiles with halo columns on
    both sides, odd and even widths."""
    rng = np.random.default_rng(70 + r)
    for H, W in [(20, 513), (17, 1100), (5, 1026)]:
        imgs = rng.integers(-1100, 400, (2, H, W)).astype(np.int16)
        _check(imgs, -1024, 3071, 256, r)


@pytest.mark.parametrize("win", [(-1024, -200, 256), (-5, 7, 13), (100, 100, 4), (-32768, 32767, 200)])
def test_open2d_windows(win):
    lo, hi, L = win
    rng = np.random.default_rng(L)
    imgs = rng.integers(lo - 30, hi + 30, (2, 50, 90)).clip(-32768, 32767).astype(np.int16)
    _check(imgs, lo, hi, L, 5)


def test_open2d_workload_slices():
    """Slices of the 300-slice workload with the paper's disk (radius 10)."""
    vol = synth.workload_volume300(0)[::100]
    _check(vol, -1024, -200, 256, 10)
    say(f"opening of {vol.shape[0]} workload slices matches the oracle")


def test_open2d_single_outputs():
    rng = np.random.default_rng(9)
    imgs = rng.integers(-1024, 500, (3, 40, 77)).astype(np.int16)
    _check(imgs, -1024, 3071, 256, 6, want=("opened",))
    _check(imgs, -1024, 3071, 256, 6, want=("residue",))
    _check(imgs, -1024, 3071, 256, 6, want=("residue16",))


@pytest.mark.parametrize("r", [2, 10])
def test_open2d_misaligned_images(r):
    """Even widths (pixel pairs load and store as one access) with images at
    odd int16 offsets of one buffer (2-byte aligned): the per-pixel path."""
    rng = np.random.default_rng(40 + r)
    H, W, n = 66, 130, 3
    buf = rng.integers(-1100, 400, n * H * W + 1).astype(np.int16)
    dbuf = to_dev(buf)
    imgs = [dbuf[1 + i * H * W: 1 + (i + 1) * H * W] for i in range(n)]
    o, res, r16 = api.open2d(api.Batch(imgs), H, W, api.binning(-1024, 3071, 256), r,
                             want=("opened", "residue", "residue16"))
    torch.cuda.synchronize()
    for i in range(n):
        g = oracle.gray(buf[1 + i * H * W: 1 + (i + 1) * H * W].reshape(H, W), -1024, 3071, 256)
        oo, rr = oracle.opening(g, r)
        assert np.array_equal(o[i].cpu().numpy().astype(np.int32), oo), (r, i)
        assert np.array_equal(res[i].cpu().numpy().astype(np.int32), rr), (r, i)
        assert np.array_equal(r16[i].cpu().numpy().astype(np.int32), rr), (r, i)


@pytest.mark.parametrize("q", [0.5, 1.5])
def test_segmentation_after_the_opening(q):
    """The paper's segmentation step on workload slices: opening by the
    disk of radius 10, then the Tsallis threshold selected on the residue
    image and the residue thresholded (histogram of its gray levels, one
    threshold, labels), all against the oracle."""
    lo, hi, L, r = -1024, -200, 256, 10
    vol = synth.workload_volume300(0)[::150]
    n, H, W = vol.shape
    _, _, r16 = api.open2d(api.Batch.slices(to_dev(vol)), H, W, api.binning(lo, hi, L), r, want=("residue16",))
    ident = api.binning(0, L - 1, L)  # each gray level its own bin
    b = api.Batch.slices(r16)
    h = api.histogram(b, ident)
    P, Q = api.prefix(h, q)
    thr, obj, st = api.threshold_search(P, Q, 1, q)
    lab = api.label(b, ident, thr, 1)
    torch.cuda.synchronize()
    Hg = h.cpu().numpy().view(np.uint32)
    for i in range(n):
        _, rr = oracle.opening(oracle.gray(vol[i], lo, hi, L), r)
        rr16 = rr.astype(np.int16)
        want_h = oracle.histogram(rr16.reshape(-1), 0, L - 1, L)
        assert np.array_equal(Hg[i], want_h), i
        check_choice(want_h, 1, q, thr[i].cpu().numpy(), obj[i].item(), st[i].item())
        want_l = oracle.label(rr16.reshape(-1), 0, L - 1, L, thr[i].cpu().numpy())
        assert np.array_equal(lab[i].cpu().numpy(), want_l), i
    say(f"segmentation after the opening, q={q}: thresholds {thr[:, 0].tolist()}")
