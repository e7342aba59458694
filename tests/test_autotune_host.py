"""Host side of the tuning ABI and of the autotuner (no GPU): the pms_tuning
layout and built-in values, null-handle rejection, the size classes, the
coordinate search and the JSON cache."""
import ctypes
import json
import os

import pytest

from paper_1708_04710_amd import _binding, api, autotune


def test_tuning_layout_defaults_and_null_handles():
    lib = _binding.load()
    assert ctypes.sizeof(_binding.PmsTuning) == 40
    t = lib.pms_default_tuning()
    assert (t.lane_blocks, t.chain_blocks, t.lane_steps, t.lane_steps_few, t.lane_many, t.lane_refill,
            t.lane_flush, t.wide_blocks, t.lane_cap, t.solve) == (2048, 512, 128, 0, 65536, 32, 16, 2048, 39, 512)
    assert api.default_tuning() == dict(lane_blocks=2048, chain_blocks=512, lane_steps=128, lane_steps_few=0,
                                        lane_many=65536, lane_refill=32, lane_flush=16, wide_blocks=2048,
                                        lane_cap=39, solve=512)
    assert lib.pms_set_tuning(None, None) == _binding.PMS_ERR_INVALID_ARG
    assert lib.pms_get_tuning(None, None) == _binding.PMS_ERR_INVALID_ARG
    assert lib.pms_autotune(None, None, 0, None, None, 0, None, None, None) == _binding.PMS_ERR_INVALID_ARG


def test_tuning_struct_overlays_the_builtin_values():
    t = api._tuning_struct(dict(lane_steps=7, lane_flush=3))
    assert (t.lane_steps, t.lane_flush, t.lane_blocks, t.wide_blocks) == (7, 3, 2048, 2048)
    with pytest.raises(KeyError):
        api._tuning_struct(dict(reserved=0))


def test_size_class_buckets():
    assert autotune.size_class(0, 0, 1) == "m0.z0.b0"
    assert autotune.size_class(1, 0, 1) == "m1.z0.b0"
    assert autotune.size_class(1023, 1024, 512) == "m10.z11.b9"
    assert autotune.size_class(1024, 1024, 513) == "m11.z11.b10"
    # the 64^3 lower-star filtration and the 64-cloud circle batch fall in different classes
    assert autotune.size_class(1_823_616 - 1, 5_000_000, 1) != autotune.size_class(2_808_832, 8_000_000, 64)
    assert autotune.cache_key("gfx950", "v", 5, 6, 2) == "gfx950/v/m3.z3.b1"


def test_coordinate_search_finds_a_separable_minimum():
    target = {"a": 3, "b": 1}
    seen = []

    def measure(cands):
        seen.append(cands)
        return [sum((c[k] - target[k]) ** 2 for k in target) for c in cands]

    best, score, scored = autotune.coordinate_search(measure, {"a": 2, "b": 2, "x": 9},
                                                     {"a": (1, 2, 3), "b": (0, 1, 2)})
    assert best == {"a": 3, "b": 1, "x": 9} and score == 0 and scored == 6
    # each call varies one parameter, the current value first
    assert [c["a"] for c in seen[0]] == [2, 1, 3] and all(c["b"] == 2 for c in seen[0])
    assert [c["b"] for c in seen[1]] == [2, 0, 1] and all(c["a"] == 3 for c in seen[1])


def test_coordinate_search_ties_keep_the_current_value():
    best, score, scored = autotune.coordinate_search(lambda cs: [1.0] * len(cs), {"a": 5, "b": 0},
                                                     {"a": (1, 2), "b": (0, 4)}, passes=3)
    assert best == {"a": 5, "b": 0} and score == 1.0 and scored == 5  # one pass: nothing changed


def test_coordinate_search_more_passes_follow_interactions():
    cost = {(0, 0): 5, (1, 0): 6, (0, 1): 4, (1, 1): 1}
    measure = lambda cs: [cost[(c["a"], c["b"])] for c in cs]
    start, grid = {"a": 0, "b": 0}, {"a": (0, 1), "b": (0, 1)}
    assert autotune.coordinate_search(measure, start, grid, passes=1)[:2] == ({"a": 0, "b": 1}, 4)
    assert autotune.coordinate_search(measure, start, grid, passes=3)[:2] == ({"a": 1, "b": 1}, 1)


def test_coordinate_search_rejects_bad_use():
    with pytest.raises(ValueError):
        autotune.coordinate_search(lambda cs: [0.0], {"a": 0}, {"a": (0, 1)})
    with pytest.raises(KeyError):
        autotune.coordinate_search(lambda cs: [0.0] * len(cs), {"a": 0}, {"b": (0, 1)})
    with pytest.raises(ValueError):
        autotune.coordinate_search(lambda cs: [0.0] * len(cs), {"a": 0}, {"a": (0, 1)}, passes=0)


def test_tune_cache_round_trip(tmp_path):
    path = tmp_path / "sub" / "tune.json"
    c = autotune.TuneCache(str(path))
    assert c.get("k") is None
    rec = {"tuning": {"lane_blocks": 768}, "graph_rounds": 4, "ms": 1.5, "scored": 6}
    c.put("k", rec)
    c.put("k2", {**rec, "graph_rounds": 0})
    assert autotune.TuneCache(str(path)).get("k") == rec
    assert sorted(os.listdir(path.parent)) == ["tune.json"]  # no temporary file left behind
    mem = autotune.TuneCache()
    mem.put("k", rec)
    assert mem.get("k") == rec
    bad = tmp_path / "bad.json"
    bad.write_text(json.dumps([1, 2]))
    with pytest.raises(ValueError):
        autotune.TuneCache(str(bad))
