"""The seeded CT-like generator: determinism and the mixture's shape."""
import numpy as np

from paper_2012_10684_amd import synth


def test_slice_deterministic_and_shaped():
    a = synth.workload_slice(0)
    b = synth.workload_slice(0)
    c = synth.workload_slice(1)
    assert a.dtype == np.int16 and a.shape == (512, 512)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= synth.HU_MIN and a.max() <= synth.HU_MAX
    # air (-1000 +- 20) is ~15 % of voxels; 11.5 % of air clips to -1024
    air = (a < -940).mean()
    assert 0.13 < air < 0.20
    assert 0.010 < (a == -1024).mean() < 0.030
    # lung : soft : bone = 45 : 30 : 10 of the rest
    soft = ((a > -100) & (a < 180)).mean()
    assert 0.26 < soft < 0.33


def test_volume_tubes_and_window_fraction():
    v = synth.make_volume(synth.rng_for(2, 99), 24, 128)
    assert v.shape == (24, 128, 128) and v.dtype == np.int16
    air = v < -940
    assert 0.13 < air.mean() < 0.22
    # tubes are continuous in z: air pixels overlap between neighbouring slices
    overlap = (air[1:] & air[:-1]).sum() / max(1, air[1:].sum())
    assert overlap > 0.5
    # about 40 % of voxels lie above -200 HU (the narrow lung window's top)
    assert 0.36 < (v > -200).mean() < 0.44


def test_batch_and_serving_recipes():
    z = synth.batch_depths(64)
    assert len(z) == 64 and min(z) >= 120 and max(z) <= 600
    tr = synth.serving_trace(50)
    assert len(tr) == 50 and all(t[2] in (256, 512) for t in tr)
    assert all(tr[i][0] <= tr[i + 1][0] for i in range(49))
