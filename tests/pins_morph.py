"""Pins of the morphology oracle (oracle/morph.c) to facts other than
itself: scipy.ndimage's gray-scale erosion and dilation with the same disk
footprint and padding that takes no part, the algebraic properties of an
opening (anti-extensive, idempotent, increasing), shapes whose opening is
known (a disk of radius >= r survives, anything too thin for the disk
vanishes), and the structuring element itself (the erosion of one dark pixel
is the disk)."""
from __future__ import annotations

import numpy as np
from scipy import ndimage

import oracle

BIG = 1 << 30


def disk(r):
    d = np.arange(-r, r + 1)
    return (d[:, None] ** 2 + d[None, :] ** 2) <= r * r


def pin_morph_equals_scipy(lib=None):
    rng = np.random.default_rng(1)
    for H, W, r in [(1, 1, 0), (5, 7, 1), (9, 4, 3), (30, 41, 5), (25, 25, 10), (6, 50, 10), (40, 33, 12)]:
        f = rng.integers(0, 256, (H, W)).astype(np.int32)
        ero = ndimage.grey_erosion(f, footprint=disk(r), mode="constant", cval=BIG)
        dil = ndimage.grey_dilation(f, footprint=disk(r), mode="constant", cval=-BIG)
        assert np.array_equal(oracle.morph(f, r, False, lib=lib), ero), (H, W, r)
        assert np.array_equal(oracle.morph(f, r, True, lib=lib), dil), (H, W, r)
        o, res = oracle.opening(f, r, lib=lib)
        want = ndimage.grey_dilation(ero, footprint=disk(r), mode="constant", cval=-BIG)
        assert np.array_equal(o, want), (H, W, r)
        assert np.array_equal(res, f - want), (H, W, r)


def pin_opening_properties(lib=None):
    rng = np.random.default_rng(2)
    for H, W, r in [(32, 48, 4), (40, 40, 10)]:
        f = rng.integers(0, 200, (H, W)).astype(np.int32)
        g = f + rng.integers(0, 40, (H, W)).astype(np.int32)  # g >= f
        of, rf = oracle.opening(f, r, lib=lib)
        og, _ = oracle.opening(g, r, lib=lib)
        assert (of <= f).all(), "opening is anti-extensive"
        assert np.array_equal(oracle.opening(of, r, lib=lib)[0], of), "opening is idempotent"
        assert (of <= og).all(), "opening is increasing"
        assert (rf >= 0).all() and np.array_equal(rf, f - of)


def pin_opening_shapes(lib=None):
    r = 6
    H = W = 48
    yy, xx = np.mgrid[:H, :W]
    # a bright union of translates of the disk (the sets an opening keeps
    # exactly) on a dark background survives unchanged
    bright = np.zeros((H, W), bool)
    for cy, cx in [(20, 18), (24, 23), (31, 26), (12, 35)]:
        bright |= (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
    f = np.where(bright, 200, 30).astype(np.int32)
    o, res = oracle.opening(f, r, lib=lib)
    assert np.array_equal(o, f) and not res.any()
    # a bright bar 2r pixels wide holds no disk of radius r (2r + 1 across): it vanishes
    f = np.full((H, W), 30, np.int32)
    f[10:40, 20:20 + 2 * r] = 200
    o, res = oracle.opening(f, r, lib=lib)
    assert (o == 30).all() and np.array_equal(res, f - 30)
    # constant image, and radius 0, leave the image unchanged
    c = np.full((H, W), 77, np.int32)
    assert np.array_equal(oracle.opening(c, r, lib=lib)[0], c)
    rnd = np.random.default_rng(3).integers(0, 256, (H, W)).astype(np.int32)
    assert np.array_equal(oracle.opening(rnd, 0, lib=lib)[0], rnd)


def pin_structuring_element(lib=None):
    """Eroding a single dark pixel in a bright field darkens exactly the disk
    of radius r around it (dx^2 + dy^2 <= r^2, boundary included)."""
    for r in (1, 2, 5, 10):
        n = 2 * r + 9
        f = np.full((n, n), 255, np.int32)
        c = n // 2
        f[c, c] = 0
        e = oracle.morph(f, r, False, lib=lib)
        d = np.arange(n) - c
        want = np.where(d[:, None] ** 2 + d[None, :] ** 2 <= r * r, 0, 255)
        assert np.array_equal(e, want), r


ALL_PINS = [pin_morph_equals_scipy, pin_opening_properties, pin_opening_shapes, pin_structuring_element]
