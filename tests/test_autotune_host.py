"""Host logic of the autotuner (no GPU): the coordinate search finds the
optimum of a separable cost from any default, keeps every trial, and the
cache round-trips a tuned configuration; apply_* call the handle's setters
with the chosen values."""
import json
import os

import pytest

from paper_1601_04633_amd import autotune


def test_coordinate_search_finds_separable_optimum():
    space = {"a": [0, 1, 2, 3], "b": ["x", "y", "z"], "c": [(1, 2), (3, 4)]}
    default = {"a": 0, "b": "x", "c": (1, 2)}
    cost_a = {0: 5.0, 1: 2.0, 2: 1.0, 3: 4.0}
    cost_b = {"x": 3.0, "y": 0.5, "z": 1.0}
    cost_c = {(1, 2): 1.0, (3, 4): 0.25}
    calls = []

    def measure(cfg):
        calls.append(dict(cfg))
        return cost_a[cfg["a"]] + cost_b[cfg["b"]] + cost_c[cfg["c"]]

    best, best_t, trials = autotune._coordinate_search(space, default, measure)
    assert best == {"a": 2, "b": "y", "c": (3, 4)}
    assert best_t == pytest.approx(1.75)
    assert len(trials) == len(calls)
    assert min(t for _, t in trials) == best_t


def test_coordinate_search_keeps_default_when_it_is_best():
    space = {"a": [0, 1, 2]}
    best, best_t, trials = autotune._coordinate_search(space, {"a": 1}, lambda c: abs(c["a"] - 1))
    assert best == {"a": 1} and best_t == 0
    assert len(trials) == 3          # the default and the two alternatives, one sweep


def test_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setattr(autotune, "CACHE_PATH", str(path))
    autotune._store_cache("k1", {"temporal": [4, 16], "sec_per_step": 1e-6})
    autotune._store_cache("k2", {"temporal": [2, 6]})
    data = json.loads(path.read_text())
    assert data["k1"]["temporal"] == [4, 16] and data["k2"]["temporal"] == [2, 6]
    assert autotune._load_cache() == data
    path.write_text("not json")
    assert autotune._load_cache() == {}


class _FakeCavity:
    def __init__(self):
        self.calls = []

    def set_launch(self, *a):
        self.calls.append(("launch", a))

    def set_temporal(self, *a):
        self.calls.append(("temporal", a))

    def set_temporal_march(self, *a):
        self.calls.append(("march", a))


class _FakeBatch:
    def __init__(self):
        self.calls = []

    def set_schedule(self, **kw):
        self.calls.append(("schedule", kw))

    def set_temporal(self, *a):
        self.calls.append(("temporal", a))

    def set_temporal_march(self, *a):
        self.calls.append(("march", a))


def test_apply_functions_call_the_setters():
    c = _FakeCavity()
    autotune.apply_cavity(c, {"temporal": (4, 12), "block": (128, 2), "xcd_remap": 0})
    assert ("launch", (128, 2, 0, 60)) in c.calls and ("temporal", (4, 12)) in c.calls
    assert all(autotune.GRAPH_STEPS % k == 0 for k in (1, 2, 3, 4, 6))
    m = _FakeCavity()
    autotune.apply_cavity(m, {"temporal": ("march", 4, 3), "block": (256, 1), "xcd_remap": 1})
    assert ("march", (4, 3, 0)) in m.calls and not any(k == "temporal" for k, _ in m.calls)
    j = _FakeCavity()                 # a configuration read back from the JSON cache
    autotune.apply_cavity(j, {"temporal": ["march", 4, 2], "block": [256, 1], "xcd_remap": 1})
    assert ("march", (4, 2, 0)) in j.calls
    b = _FakeBatch()
    autotune.apply_batch(b, {"temporal": (3, 16), "block": (64, 4), "order": 2, "grid_blocks": 4096,
                             "group": (96 << 20, 8)})
    assert b.calls[0] == ("schedule", dict(block_x=64, block_y=4, order=2, grid_blocks=4096,
                                           group_bytes=96 << 20, group_steps=8))
    assert b.calls[1] == ("temporal", (3, 16))
    bm = _FakeBatch()                 # the marching form, as read back from the JSON cache
    autotune.apply_batch(bm, {"temporal": ["march", 6, 2], "block": [64, 4], "order": 1, "grid_blocks": 0,
                              "group": [0, 64]})
    assert bm.calls[1] == ("march", (6, 2, 0)) and not any(k == "temporal" for k, _ in bm.calls)


def test_search_spaces_only_hold_supported_pairs():
    """Every steps-per-launch pair the tuner may try is one the library
    accepts (the header's list for dmrt_set_temporal)."""
    ok = {(1, 4), (1, 6), (1, 10), (1, 16), (2, 4), (2, 6), (2, 10), (2, 16), (3, 6), (3, 10), (3, 12),
          (3, 14), (3, 16), (4, 10), (4, 12), (4, 14), (4, 16)}
    march_ok = {(2, 8), (3, 2), (3, 4), (4, 1), (4, 2), (4, 3), (4, 4), (6, 2)}   # dmrt_set_temporal_march
    for kr in autotune.ADJOINT_SPACE:
        assert tuple(kr) in ok, kr
    for kr in autotune.CAVITY_SPACE["temporal"] + autotune.BATCH_SPACE["temporal"]:
        if kr[0] == "march":
            assert tuple(kr[1:3]) in march_ok, kr
        else:
            assert tuple(kr) in ok, kr


def test_host_timer_waits_for_the_handle():
    """Without a stream pointer the timer uses host time and calls the
    handle's synchronisation before reading it, so queued work is counted."""
    calls = []
    start, stop = autotune._timer(None, lambda: calls.append(1))
    start()
    t = stop()
    assert calls == [1] and t >= 0
