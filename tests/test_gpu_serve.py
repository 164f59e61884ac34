"""Serving engine on the GPU: a request's result is the same, bit for bit,
whether it is served alone or batched with others, and matches the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import check_choice, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2012_10684_amd import api, synth  # noqa: E402
from paper_2012_10684_amd.serve import Engine, Request, latency_stats  # noqa: E402

LO, HI, L, K, QS = -1024, 3071, 512, 3, (0.8, 1.5)


@pytest.fixture(scope="module")
def volumes():
    """Requests of uneven sizes (some not a multiple of 8 voxels)."""
    shapes = [(7, 96, 96), (3, 256, 256), (11, 64, 61), (1, 128, 128), (5, 200, 150), (9, 96, 96), (2, 256, 255)]
    return [synth.make_volume(synth.rng_for(5, 900 + i), z, max(h, w))[:, :h, :w].copy()
            for i, (z, h, w) in enumerate(shapes)]


def _alone(vol):
    dv = to_dev(vol.reshape(-1))
    b = api.Batch([dv])
    binn = api.binning(LO, HI, L)
    h = api.histogram(b, binn)
    P, Q = api.prefix(h, QS)
    thr, obj, st = api.threshold_search(P, Q, K, QS)
    labs = api.label_sets(b, binn, [thr[j] for j in range(len(QS))], K)
    torch.cuda.synchronize()
    return thr[:, 0].cpu().numpy(), obj[:, 0].cpu().numpy(), st[:, 0].cpu().numpy(), [l[0].cpu() for l in labs]


@pytest.mark.parametrize("max_batch_voxels,max_inflight", [(1 << 30, 2), (200_000, 2), (1, 1)],
                         ids=["one-batch", "several", "serial"])
def test_engine_batched_equals_alone(volumes, max_batch_voxels, max_inflight):
    eng = Engine(api.binning(LO, HI, L), K, QS, max_batch_voxels=max_batch_voxels, max_inflight=max_inflight)
    reqs = [Request(i, torch.from_numpy(v).pin_memory(), 0.0) for i, v in enumerate(volumes)]
    say(f"engine: {len(reqs)} requests, max_batch_voxels={max_batch_voxels}")
    res = {r.rid: r for r in eng.run(reqs, realtime=False)}
    assert sorted(res) == list(range(len(volumes)))
    for i, v in enumerate(volumes):
        thr, obj, st, labs = _alone(v)
        r = res[i]
        assert np.array_equal(r.thr, thr) and np.array_equal(r.status, st), i
        assert np.array_equal(r.obj, obj, equal_nan=True), i
        for j in range(len(QS)):
            assert torch.equal(r.labels[j], labs[j]), (i, j)
    # the oracle on the two smallest requests
    for i in (3, 2):
        h = oracle.histogram(volumes[i], LO, HI, L)
        for j, q in enumerate(QS):
            check_choice(h, K, q, res[i].thr[j], res[i].obj[j], int(res[i].status[j]))
            want = oracle.label(volumes[i].reshape(-1), LO, HI, L, res[i].thr[j])
            assert np.array_equal(res[i].labels[j].numpy(), want)


def test_engine_realtime_trace(volumes):
    """Arrivals spread in time, label buffers from the pinned pool given back
    as each result is seen: every result is still bit-identical to the
    request served alone, and the device-side times are measured."""
    nmax = max(v.size for v in volumes)
    eng = Engine(api.binning(LO, HI, L), K, QS, max_batch_voxels=300_000, max_request_voxels=nmax, pool_slots=64)
    reqs = [Request(i, torch.from_numpy(volumes[i % len(volumes)]).pin_memory(), 0.004 * i) for i in range(20)]
    alone = {i: _alone(v) for i, v in enumerate(volumes)}
    checked = []

    def check(r):
        thr, obj, st, labs = alone[r.rid % len(volumes)]
        assert r.error is None and np.array_equal(r.thr, thr) and np.array_equal(r.status, st), r.rid
        for j in range(len(QS)):
            assert torch.equal(r.labels[j], labs[j]), (r.rid, j)
        checked.append(r.rid)
        eng.release(r)  # the buffers go back to the pool

    res = eng.run(reqs, realtime=True, on_result=check)
    assert sorted(checked) == list(range(20))
    for r in res:
        assert r.done >= r.admitted >= r.arrival - 1e-9
        assert 0 < r.kernels_s <= r.device_s <= r.done - r.admitted + 1e-3
    st = latency_stats(res, wall=max(r.done for r in res))
    say(f"realtime trace: {st}; pinned buffers allocated outside the pool: {eng.backend.pool.extra}")
    assert st["p99_s"] >= st["p50_s"] > 0 and st["device_p99_s"] >= st["device_p50_s"] > 0
    assert eng.backend.pool.extra == 0


def test_engine_serving_size_requests_against_the_oracle():
    """Requests of the serving workload's sizes (512x512x300 and 256x256x200
    volumes, whole-volume 512-bin histograms over [-1024, 3071], k = 3,
    q = 0.8) served together: thresholds, objectives and every label against
    the oracle."""
    vols = [synth.serving_volume(700, 300, 512), synth.serving_volume(701, 200, 256)]
    eng = Engine(api.binning(LO, HI, L), K, (0.8,))
    reqs = [Request(i, torch.from_numpy(v).pin_memory(), 0.0) for i, v in enumerate(vols)]
    say(f"engine: serving-size requests {[v.shape for v in vols]}")
    res = {r.rid: r for r in eng.run(reqs, realtime=False)}
    for i, v in enumerate(vols):
        h = oracle.histogram(v, LO, HI, L)
        assert int(h.sum()) == v.size
        exact, ref = check_choice(h, K, 0.8, res[i].thr[0], res[i].obj[0], int(res[i].status[0]))
        say(f"request {i} {v.shape}: thresholds {res[i].thr[0].tolist()} (oracle {ref.thr.tolist()}, "
            f"runner-up gap {ref.rel_gap():.2e})")
        want = oracle.label(v.reshape(-1), LO, HI, L, res[i].thr[0])
        assert np.array_equal(res[i].labels[0].numpy(), want), i
