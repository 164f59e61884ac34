"""GPU parity on the five workloads at their full sizes, in the launch
configuration the benchmark times, against the oracle (all outputs where the
oracle finishes in seconds, sampled problems otherwise)."""
import numpy as np
import pytest

import oracle
from gpu_util import check_choice, say, to_dev, u32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2012_10684_amd import api, synth  # noqa: E402


def test_single_slice_4096_bins_k1():
    """One 512x512 slice, 4096 bins over [-1024, 3071], k = 1, q = 0.8."""
    for idx in range(3):
        s = synth.workload_slice(idx)
        binn = api.binning(-1024, 3071, 4096)
        h, (thr, obj, st), labels = api.segment(api.Batch([to_dev(s.reshape(-1))]), binn, 1, 0.8)
        labels = labels[0]
        torch.cuda.synchronize()
        hh = oracle.histogram(s, -1024, 3071, 4096)
        assert np.array_equal(u32(h)[0], hh)
        exact, r = check_choice(hh, 1, 0.8, thr.cpu().numpy()[0], float(obj[0]), int(st[0]))
        say(f"slice {idx}: gpu {thr.cpu().numpy()[0].tolist()} oracle {r.thr.tolist()} gap {r.rel_gap():.3g}")
        want = oracle.label(s.reshape(-1), -1024, 3071, 4096, r.thr if exact else thr.cpu().numpy()[0])
        assert np.array_equal(labels[0].cpu().numpy(), want)


@pytest.fixture(scope="module")
def volume300():
    say("generating the 512x512x300 volume")
    return synth.workload_volume300(0)


@pytest.mark.parametrize("q", [0.5, 0.8, 1.5])
def test_volume300_per_slice_k2(volume300, q):
    """Per-slice 256-bin histograms over [-1024, -200], k = 2, every slice."""
    vol = volume300
    dv = to_dev(vol)
    b = api.Batch.slices(dv)
    binn = api.binning(-1024, -200, 256)
    h, (thr, obj, st), labels = api.segment(b, binn, 2, q)
    labels = labels[0]
    torch.cuda.synchronize()
    H = u32(h)
    thr, obj, st = thr.cpu().numpy(), obj.cpu().numpy(), st.cpu().numpy()
    exact = 0
    for z in range(vol.shape[0]):
        hz = oracle.histogram(vol[z], -1024, -200, 256)
        assert np.array_equal(H[z], hz), z
        ex, r = check_choice(hz, 2, q, thr[z], obj[z], st[z])
        exact += ex
        if z % 50 == 0:
            lab = labels[z].cpu().numpy()
            assert np.array_equal(lab, oracle.label(vol[z].reshape(-1), -1024, -200, 256, thr[z]))
    say(f"q={q}: {exact}/{vol.shape[0]} slices with identical thresholds")
    # every label, against the oracle's labels for the GPU thresholds (which
    # the loop above showed to be the oracle's choice up to the tie rule)
    allv = vol.reshape(vol.shape[0], -1)
    for z in range(vol.shape[0]):
        want = oracle.label(allv[z], -1024, -200, 256, thr[z])
        assert np.array_equal(labels[z].cpu().numpy(), want), z


def test_volume600_whole_k3():
    """Whole-volume 1024-bin histogram of 512x512x600, k = 3, q = 0.8."""
    say("generating the 512x512x600 volume")
    vol = synth.workload_volume600(0)
    dv = to_dev(vol)
    b = api.Batch([dv.reshape(-1)])
    binn = api.binning(-1024, 3071, 1024)
    h, (thr, obj, st), labels = api.segment(b, binn, 3, 0.8)
    labels = labels[0]
    torch.cuda.synchronize()
    hh = oracle.histogram(vol, -1024, 3071, 1024)
    assert np.array_equal(u32(h)[0], hh)
    say("oracle search k=3 L=1024")
    ex, r = check_choice(hh, 3, 0.8, thr.cpu().numpy()[0], float(obj[0]), int(st[0]))
    say(f"gpu {thr.cpu().numpy()[0].tolist()} oracle {r.thr.tolist()} S {float(obj[0])!r} vs {r.obj!r}")
    want = oracle.label(vol.reshape(-1), -1024, 3071, 1024, thr.cpu().numpy()[0])
    assert np.array_equal(labels[0].cpu().numpy(), want)


def test_batch64_full_size():
    """64 volumes 512x512xU{120..600} (about 23,000 slices, 6e9 voxels), each
    generated separately with its own tissue fractions (worker processes),
    in one batch: per-slice 256 bins over [-1024, -200], k = 2, q in {0.5,
    0.8, 1.5}, labels for every q in one pass -- the benchmark's launch
    configuration.  Every slice: counts sum to its voxels, a valid ascending
    tuple, and label counts equal to its histogram's class masses at the
    chosen thresholds (a property of the labels that holds at any size).
    Four slices of every volume (first, last and two drawn at random):
    histograms, thresholds, objectives and labels against the oracle."""
    depths = synth.batch_depths(64)
    say(f"generating 64 volumes ({sum(depths)} slices) in worker processes")
    pool, it = synth.generate_parallel(list(enumerate(depths)), workers=12)
    rng = np.random.default_rng(64)
    dvols, picks = [], []
    base = 0
    for i, v in enumerate(it):
        assert v.shape == (depths[i], 512, 512)
        dvols.append(to_dev(v))
        zs = sorted({0, depths[i] - 1} | set(rng.integers(1, depths[i] - 1, 2).tolist()))
        picks += [(base + z, v[z].reshape(-1).copy()) for z in zs]
        base += depths[i]
        del v
    pool.close()
    pool.join()
    S = 512 * 512
    segs = [v[z].reshape(-1) for v in dvols for z in range(v.shape[0])]
    b = api.Batch(segs)
    nseg = b.nseg
    binn = api.binning(-1024, -200, 256)
    qs = (0.5, 0.8, 1.5)
    flat = [torch.empty((nseg, S), dtype=torch.uint8, device=dvols[0].device) for _ in qs]  # labels, slice-major
    outs = [[f[i] for i in range(nseg)] for f in flat]
    h = api.histogram(b, binn, tune="auto")
    P, Q = api.prefix(h, qs)
    thr, obj, st = api.threshold_search(P, Q, 2, qs, tune="auto")
    api.label_sets(b, binn, [thr[j] for j in range(3)], 2, outs=outs, tune="auto")
    torch.cuda.synchronize()
    say(f"{nseg} slices segmented; checking every slice's invariants")
    assert int((st != 0).sum()) == 0
    hc = h.to(torch.int64)
    assert bool((hc.sum(dim=1) == S).all())
    t = thr.to(torch.int64)  # [nq, nseg, 2]
    assert bool(((t[..., 0] >= 0) & (t[..., 0] < t[..., 1]) & (t[..., 1] <= 254)).all())
    cum = hc.cumsum(dim=1)  # counts of bins <= t
    for j in range(3):
        c0 = cum.gather(1, t[j, :, :1])[:, 0]
        c1 = cum.gather(1, t[j, :, 1:])[:, 0]
        for lab, want in ((0, c0), (1, c1 - c0), (2, S - c1)):
            got = (flat[j] == lab).sum(dim=1)
            assert torch.equal(got, want), (j, lab, int((got != want).sum()))
    say(f"checking {len(picks)} slices against the oracle")
    H = u32(h)
    thr_h, obj_h, st_h = thr.cpu().numpy(), obj.cpu().numpy(), st.cpu().numpy()
    for i, sl in picks:
        want_h = oracle.histogram(sl, -1024, -200, 256)
        assert np.array_equal(H[i], want_h), i
        for j, q in enumerate(qs):
            check_choice(want_h, 2, q, thr_h[j, i], obj_h[j, i], st_h[j, i])
            want = oracle.label(sl, -1024, -200, 256, thr_h[j, i])
            assert np.array_equal(flat[j][i].cpu().numpy(), want), (i, q)
    # the benchmark's launch: q = 0.8 through ts_segment (one workgroup per
    # slice, the whole path in one launch): every output bit-identical to the
    # separate passes above
    say("the same batch at q = 0.8 through ts_segment")
    fl = torch.empty((nseg, S), dtype=torch.uint8, device=dvols[0].device)
    hf, (tf, of, sf), _ = api.segment(b, binn, 2, 0.8, label_outs=[[fl[i] for i in range(nseg)]], tune="auto")
    torch.cuda.synchronize()
    assert torch.equal(hf, h)
    assert torch.equal(tf, thr[1]) and torch.equal(sf, st[1])
    assert torch.equal(of.view(torch.int64), obj[1].view(torch.int64))
    assert torch.equal(fl, flat[1])
