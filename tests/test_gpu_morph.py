"""GPU parity of the morphology step (ts_open2d) against the oracle: the
opened image and the residue gray - opened bit-exact, for radii 0..32,
images smaller than a tile or than the disk, sizes that leave ragged tiles,
narrow and wide windows, CT-like slices of the workload, and each output
requested alone."""
import numpy as np
import pytest

import oracle
from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2012_10684_amd import api, synth  # noqa: E402


def _check(imgs, lo, hi, L, r, want=("opened", "residue")):
    n, H, W = imgs.shape
    dv = to_dev(imgs)
    o, res = api.open2d(api.Batch.slices(dv), H, W, api.binning(lo, hi, L), r, want=want)
    torch.cuda.synchronize()
    for i in range(n):
        g = oracle.gray(imgs[i], lo, hi, L)
        oo, rr = oracle.opening(g, r)
        if o is not None:
            assert np.array_equal(o[i].cpu().numpy().astype(np.int32), oo), (H, W, r, i)
        if res is not None:
            assert np.array_equal(res[i].cpu().numpy().astype(np.int32), rr), (H, W, r, i)


@pytest.mark.parametrize("r", [0, 1, 3, 10, 17, 32])
def test_open2d_random_images(r):
    rng = np.random.default_rng(r + 1)
    for H, W in [(1, 1), (3, 200), (64, 64), (70, 129), (130, 65)]:
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
