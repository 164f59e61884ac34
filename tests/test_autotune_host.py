"""Tuning lookup of ts_segment (CPU): a call without its own cache entry takes
the cached shapes of the separate steps it may run (histogram, search of
nseg x nq problems, labels of nq sets), merged; its own entry wins."""
import json

import pytest

from paper_2012_10684_amd import api, autotune


@pytest.fixture()
def cache(tmp_path, monkeypatch):
    def use(entries):
        p = tmp_path / "tuned.json"
        p.write_text(json.dumps({k: {"tuning": v, "us": 1.0} for k, v in entries.items()}))
        monkeypatch.setenv("TS_AUTOTUNE_CACHE", str(p))
        monkeypatch.setattr(autotune, "_default", None)
    return use


def test_segment_merges_the_steps(cache):
    nseg, total, L, k, nq, mode = 300, 300 * 512 * 512, 256, 2, 3, api.SEARCH_FP32_TIECHECK
    cache({autotune.key_histogram(nseg, total, L): {"hist_block": 1024, "hist_replicas": 16},
           autotune.key_search(nseg * nq, L, k, mode): {"search_cols": 1, "search_rows": 32},
           autotune.key_label(nseg, total, k, nq): {"label_block": 256, "label_vecs": 4},
           autotune.key_label(nseg, total, k): {"label_block": 128}})  # one set: not this call's
    got = autotune.lookup_segment(nseg, total, L, k, nq, mode)
    assert got == {"hist_block": 1024, "hist_replicas": 16, "search_cols": 1, "search_rows": 32,
                   "label_block": 256, "label_vecs": 4}
    t = api.Tuning.from_dict(got)
    assert (t.hist_block, t.search_rows, t.label_vecs) == (1024, 32, 4)


def test_segment_own_entry_wins_and_none_without_entries(cache):
    nseg, total, L, k, nq, mode = 20000, 6 * 10 ** 9, 256, 2, 1, api.SEARCH_FP32_TIECHECK
    cache({autotune.key_segment(nseg, total, L, k, nq): {"segment_block": 256},
           autotune.key_histogram(nseg, total, L): {"hist_block": 512}})
    assert autotune.lookup_segment(nseg, total, L, k, nq, mode) == {"segment_block": 256}
    cache({})
    assert autotune.lookup_segment(nseg, total, L, k, nq, mode) is None
