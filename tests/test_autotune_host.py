"""The autotuner's choice among timed candidates (no GPU): of the candidates
within the margin of the fastest, the one closest to the library defaults."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_1612_06257_amd import autotune  # noqa: E402

DEFAULTS = {"long_ring": 72, "waves_per_cu": 4, "lane4_min_bytes": 128, "use_graph": 0,
            "isolate_long": 1}


def _bucketed(**kw):
    return dict(dict(DEFAULTS, **kw), path="bucketed")


def test_candidate_set_is_the_documented_one():
    cands = list(autotune.candidates())
    bucketed = [c for c in cands if c["path"] == "bucketed"]
    assert len(bucketed) == 72 and len(cands) == 74
    assert all(c["waves_per_cu"] == 4 for c in bucketed if c["isolate_long"])
    assert _bucketed() in cands


def test_distance_counts_changed_settings():
    assert autotune.distance(_bucketed(), DEFAULTS) == 0
    assert autotune.distance(_bucketed(long_ring=96, lane4_min_bytes=0), DEFAULTS) == 2
    assert autotune.distance({"path": "lane4"}, DEFAULTS) == len(autotune.TUNING_KEYS) + 1


def test_defaults_kept_within_the_margin():
    res = [(1.000, _bucketed()), (0.997, _bucketed(long_ring=96)), (1.5, {"path": "lane4"})]
    sec, best, default = autotune.pick(res, DEFAULTS, margin=0.005)
    assert best == _bucketed() and sec == 1.000 and default == 1.000


def test_closest_of_the_near_ties_wins():
    # two settings beat the defaults clearly and tie with each other: the one
    # that changes fewer settings is kept, even if it timed slower
    res = [(1.000, _bucketed()), (0.990, _bucketed(lane4_min_bytes=0)),
           (0.988, _bucketed(lane4_min_bytes=0, long_ring=96))]
    sec, best, default = autotune.pick(res, DEFAULTS, margin=0.005)
    assert best == _bucketed(lane4_min_bytes=0) and sec == 0.990 and default == 1.000


def test_clearly_faster_candidate_wins():
    res = [(1.000, _bucketed()), (0.900, _bucketed(waves_per_cu=8, isolate_long=0)),
           (0.950, {"path": "lane1"})]
    sec, best, _ = autotune.pick(res, DEFAULTS, margin=0.005)
    assert best == _bucketed(waves_per_cu=8, isolate_long=0) and sec == 0.900


def test_fastest_wins_when_defaults_were_not_timed():
    res = [(1.000, _bucketed(long_ring=48)), (0.990, _bucketed(long_ring=96))]
    sec, best, default = autotune.pick(res, DEFAULTS, margin=0.005)
    assert best["long_ring"] == 96 and default is None


def test_zero_margin_is_the_plain_minimum():
    res = [(1.000, _bucketed()), (0.999, _bucketed(long_ring=96))]
    assert autotune.pick(res, DEFAULTS, margin=0.0)[1]["long_ring"] == 96


def test_no_candidates_is_an_error():
    with pytest.raises(ValueError):
        autotune.pick([], DEFAULTS)
