"""Seeded synthetic CT-like int16 volumes (numpy only).

The paper's patient chest CT is not public, so every input here is drawn from
a four-tissue Hounsfield-unit mixture with airway lumen structure.  This module
is shared by the GPU tests, the benchmark and the oracle tests; it holds none
of the thresholding method's arithmetic (no bin map, histogram or entropy).

Recipe (generator version ``GEN_VERSION``):
  * tissues (HU mean, std, fraction): air (-1000, 20, 15 %), lung (-850, 60,
    45 %), soft tissue (40, 40, 30 %), bone (700, 200, 10 %);
  * air voxels are placed spatially: lumen discs of radius U{3..12} px in a
    single slice, or 3-D branching tubes whose centres follow random walks
    from slice to slice in a volume; discs/tubes are added until the air
    fraction reaches the target;
  * every other voxel draws lung : soft : bone in the ratio of their
    fractions;
  * HU = clip(rint(mean + std * z), -1024, 3071) -> int16 (round half even);
  * RNG: numpy PCG64 seeded by SeedSequence([20121068, config, index]).
"""
from __future__ import annotations

import numpy as np

GEN_VERSION = 1
SEED_BASE = 20121068
HU_MIN, HU_MAX = -1024, 3071

# (name, mean HU, std HU, fraction of voxels)
TISSUES = (
    ("air", -1000.0, 20.0, 0.15),
    ("lung", -850.0, 60.0, 0.45),
    ("soft", 40.0, 40.0, 0.30),
    ("bone", 700.0, 200.0, 0.10),
)
R_MIN, R_MAX = 3, 12

_DISC = {}


def rng_for(config: int, index: int = 0) -> np.random.Generator:
    """The generator for volume ``index`` of workload ``config``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, int(config), int(index)])))


def _disc(r: int):
    if r not in _DISC:
        d = np.arange(-r, r + 1)
        dy, dx = np.meshgrid(d, d, indexing="ij")
        m = dy * dy + dx * dx <= r * r
        _DISC[r] = (dy[m].astype(np.int64), dx[m].astype(np.int64))
    return _DISC[r]


def _stamp(mask2d: np.ndarray, cy, cx, rr):
    """Set every pixel within radius rr of (cy, cx) in a 2-D mask."""
    H, W = mask2d.shape
    for r in np.unique(rr):
        sel = rr == r
        dy, dx = _disc(int(r))
        ys = cy[sel][:, None] + dy[None, :]
        xs = cx[sel][:, None] + dx[None, :]
        ok = (ys >= 0) & (ys < H) & (xs >= 0) & (xs < W)
        mask2d[ys[ok], xs[ok]] = True


def _fractions(scale=None):
    f = np.array([t[3] for t in TISSUES], dtype=np.float64)
    if scale is not None:
        f = f * np.asarray(scale, dtype=np.float64)
    return f / f.sum()


def _fill(rng: np.random.Generator, air: np.ndarray, frac: np.ndarray) -> np.ndarray:
    """Draw HU values: air where the mask is set, else lung/soft/bone."""
    n = air.size
    mu = np.array([t[1] for t in TISSUES], dtype=np.float32)
    sd = np.array([t[2] for t in TISSUES], dtype=np.float32)
    rest = frac[1:] / frac[1:].sum()
    cum = np.cumsum(rest)[:-1].astype(np.float32)
    u = rng.random(n, dtype=np.float32)
    cls = np.ones(n, dtype=np.int8)
    for c in cum:
        cls += u >= c
    cls[air.reshape(-1)] = 0
    z = rng.standard_normal(n, dtype=np.float32)
    v = mu[cls] + sd[cls] * z
    v = np.rint(v)
    np.clip(v, HU_MIN, HU_MAX, out=v)
    return v.astype(np.int16).reshape(air.shape)


def make_slice(rng: np.random.Generator, size: int = 512, frac_scale=None) -> np.ndarray:
    """One size x size slice with circular lumen discs (radius U{3..12})."""
    frac = _fractions(frac_scale)
    target = frac[0]
    air = np.zeros((size, size), dtype=bool)
    while air.mean() < target:
        nb = 16
        rr = rng.integers(R_MIN, R_MAX + 1, nb)
        cy = rng.integers(0, size, nb)
        cx = rng.integers(0, size, nb)
        _stamp(air, cy, cx, rr)
    return _fill(rng, air, frac)


def _tube_discs(rng: np.random.Generator, Z: int, size: int, est_area: float):
    """Random-walk branching tubes; returns disc records (z, y, x, r) whose
    summed area (ignoring overlap) reaches est_area."""
    zs, ys, xs, rs = [], [], [], []
    area = 0.0
    while area < est_area:
        r = int(rng.integers(R_MIN, R_MAX + 1))
        z0 = int(rng.integers(0, Z))
        length = int(rng.integers(max(1, Z // 4), Z + 1))
        stack = [(z0, float(rng.uniform(r, size - r)), float(rng.uniform(r, size - r)), r, length)]
        while stack and area < est_area:
            z, y, x, r, length = stack.pop()
            for _ in range(length):
                if z >= Z:
                    break
                zs.append(z)
                ys.append(int(round(y)))
                xs.append(int(round(x)))
                rs.append(r)
                area += np.pi * r * r
                y = min(max(y + rng.normal(0.0, 1.0), 0.0), size - 1.0)
                x = min(max(x + rng.normal(0.0, 1.0), 0.0), size - 1.0)
                z += 1
                if r > R_MIN and rng.random() < 0.02:  # branch
                    rc = int(max(R_MIN, r - rng.integers(1, 4)))
                    stack.append((z, y, x, rc, int(rng.integers(max(1, Z // 8), Z // 2 + 2))))
    return (np.asarray(zs, np.int64), np.asarray(ys, np.int64), np.asarray(xs, np.int64), np.asarray(rs, np.int64))


def make_volume(rng: np.random.Generator, Z: int, size: int = 512, frac_scale=None,
                chunk: int = 16) -> np.ndarray:
    """A Z x size x size volume with 3-D branching lumen tubes."""
    frac = _fractions(frac_scale)
    target = frac[0]
    air = np.zeros((Z, size, size), dtype=bool)
    budget = target * Z * size * size
    got = 0.0
    for _ in range(64):
        zs, ys, xs, rs = _tube_discs(rng, Z, size, (budget - got) * 1.15 + 1.0)
        order = np.argsort(zs, kind="stable")
        zs, ys, xs, rs = zs[order], ys[order], xs[order], rs[order]
        bounds = np.searchsorted(zs, np.arange(Z + 1))
        for z in range(Z):
            a, b = bounds[z], bounds[z + 1]
            if b > a:
                _stamp(air[z], ys[a:b], xs[a:b], rs[a:b])
        got = float(air.sum())
        if got >= budget:
            break
    out = np.empty((Z, size, size), dtype=np.int16)
    for z0 in range(0, Z, chunk):
        z1 = min(Z, z0 + chunk)
        out[z0:z1] = _fill(rng, air[z0:z1], frac)
    return out


# ----------------------------------------------------------------------------
# The five workloads.  Each returns host int16 arrays (C order).

def workload_slice(index: int = 0) -> np.ndarray:
    """One 512x512 slice (single-threshold, 4096-bin workload)."""
    return make_slice(rng_for(1, index), 512)


def workload_volume300(index: int = 0) -> np.ndarray:
    """One 512x512x300 volume (per-slice 256-bin, k=2 workload)."""
    return make_volume(rng_for(2, index), 300, 512)


def workload_volume600(index: int = 0) -> np.ndarray:
    """One 512x512x600 volume (whole-volume 1024-bin, k=3 workload)."""
    return make_volume(rng_for(3, index), 600, 512)


def batch_depths(count: int = 64, seed_index: int = 0):
    """Slice counts of the batched workload: Z ~ U{120..600} per volume."""
    rng = rng_for(4, 10_000 + seed_index)
    return [int(z) for z in rng.integers(120, 601, count)]


def workload_batch_volume(index: int, Z: int, size: int = 512) -> np.ndarray:
    """Volume ``index`` of the batched workload: tissue fractions scaled by
    U(0.9, 1.1) each, then renormalised."""
    rng = rng_for(4, index)
    scale = rng.uniform(0.9, 1.1, 4)
    return make_volume(rng, Z, size, frac_scale=scale)


def batch_volume_job(job) -> np.ndarray:
    """Worker entry of generate_parallel: job = (index, Z) of a batched
    workload volume."""
    i, z = job
    return workload_batch_volume(i, z)


def generate_parallel(jobs, workers: int = 0, fn=batch_volume_job):
    """Start worker processes (spawned, numpy only) that build fn(job) for
    every job; returns the pool and an iterator over the results in job order,
    each delivered as soon as it and the ones before it are done.  Call
    close() and join() on the pool afterwards."""
    import multiprocessing as mp
    import os

    n = workers or max(1, min(16, len(os.sched_getaffinity(0))))
    pool = mp.get_context("spawn").Pool(max(1, min(n, len(jobs))))
    return pool, pool.imap(fn, jobs)


def serving_trace(count: int = 600, rate: float = 20.0, seed_index: int = 0):
    """Poisson arrivals: list of (arrival_s, Z, size); sizes 50/50 small
    (256x256xU{60..300}) or large (512x512xU{120..600})."""
    rng = rng_for(5, 10_000 + seed_index)
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        if rng.random() < 0.5:
            out.append((float(t[i]), int(rng.integers(60, 301)), 256))
        else:
            out.append((float(t[i]), int(rng.integers(120, 601)), 512))
    return out


def serving_volume(index: int, Z: int, size: int) -> np.ndarray:
    return make_volume(rng_for(5, index), Z, size)
