"""Host logic of the launch-shape autotuner: candidate lists and the cache."""
import json

import pytest

at = pytest.importorskip("paper_2007_05718_amd.autotune")


def test_candidates_default_first_unique_and_clipped():
    d = at.Tiling(64, 1, 32, 8)
    c = at.candidate_tilings(256, 256, 20, d)
    assert c[0] == d
    assert len({t.as_tuple() for t in c}) == len(c)
    assert all(t.zlen <= 20 for t in c[1:])
    assert all(t.tx * t.ty == 64 for t in c)
    assert len(c) <= 24


def test_candidates_skip_tiles_wider_than_the_row():
    c = at.candidate_tilings(12, 40, 64, None)
    assert {t.tx for t in c} == {8, 16}
    c = at.candidate_tilings(5, 5, 5, None)
    assert {t.tx for t in c} == {8}
    assert {t.zlen for t in c} == {5}


def test_bad_tile_rejected():
    with pytest.raises(ValueError):
        at.candidate_tilings(64, 64, 64, None, tiles=((32, 4),))


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    cache = at.TuningCache(path)
    rep = at.TuneReport(best=at.Tiling(32, 2, 16, 4), best_ms=1.5,
                        default=at.Tiling(64, 1, 32, 8), default_ms=2.0)
    assert rep.speedup == pytest.approx(2.0 / 1.5)
    cache.put("k1", rep)
    again = at.TuningCache(path)
    assert again.get("k1") == at.Tiling(32, 2, 16, 4)
    assert again.get("missing") is None
    assert json.load(open(path))["k1"]["default_ms"] == 2.0
