"""The launch-shape tuner on a synthetic cost function (no GPU): coordinate search order, the
margin below which the held value stays, and the per-workload caches."""
import json

import pytest

from paper_2511_08929_amd import autotune

SPACE = {"a": (1, 2, 4), "b": (10, 20)}


def _cost(table):
    calls = []

    def run(cfg):
        calls.append((cfg["a"], cfg["b"]))
        return table[(cfg["a"], cfg["b"])]
    return run, calls


@pytest.fixture(autouse=True)
def _fresh(monkeypatch):
    monkeypatch.setattr(autotune, "_memory", {})
    monkeypatch.setattr(autotune, "device_key", lambda: "testdev|0|0")


def test_coordinate_search_takes_clear_improvements():
    t = {(1, 10): 1.0, (2, 10): 0.8, (4, 10): 0.9, (1, 20): 1.0, (2, 20): 0.5, (4, 20): 0.7}
    run, calls = _cost(t)
    best, timings, cached = autotune.tune("w", run, space=SPACE, start={"a": 1, "b": 10})
    assert best == {"a": 2, "b": 20} and not cached
    # a is swept with b held at 10, then b with a held at 2; no configuration is timed twice
    assert calls == [(1, 10), (2, 10), (4, 10), (2, 20)]
    assert len(timings) == len(calls)


def test_held_value_kept_within_margin():
    t = {(1, 10): 1.000, (2, 10): 0.995, (4, 10): 1.2, (1, 20): 0.98, (2, 20): 0.9, (4, 20): 1.3}
    run, _ = _cost(t)
    best, _, _ = autotune.tune("w", run, space=SPACE, start={"a": 1, "b": 10}, margin=0.01)
    assert best == {"a": 1, "b": 20}           # 0.5% faster a=2 is noise; b=20 is 2% faster
    autotune._memory.clear()
    best0, _, _ = autotune.tune("w", run, space=SPACE, start={"a": 1, "b": 10}, margin=0.0)
    assert best0 == {"a": 2, "b": 20}


def test_start_value_outside_the_space_is_timed_and_can_stay():
    t = {(3, 10): 0.5, (1, 10): 1.0, (2, 10): 0.9, (4, 10): 0.7, (3, 20): 0.6}
    run, calls = _cost(t)
    best, _, _ = autotune.tune("w", run, space=SPACE, start={"a": 3, "b": 10})
    assert best == {"a": 3, "b": 10} and calls[0] == (3, 10)


def test_results_cached_in_memory_and_on_disk(tmp_path):
    t = {(a, b): a + b / 100 for a in (1, 2, 4) for b in (10, 20)}
    run, calls = _cost(t)
    path = str(tmp_path / "tune.json")
    best, _, cached = autotune.tune("w1", run, space=SPACE, cache_path=path, start={"a": 4, "b": 20})
    assert best == {"a": 1, "b": 10} and not cached
    n = len(calls)
    again, _, cached = autotune.tune("w1", run, space=SPACE, cache_path=path)
    assert again == best and cached and len(calls) == n
    autotune._memory.clear()                   # a new process: read back from the file
    again, _, cached = autotune.tune("w1", run, space=SPACE, cache_path=path)
    assert again == best and cached and len(calls) == n
    data = json.load(open(path))
    assert [v["workload"] for v in data.values()] == ["w1"]
    other, _, cached = autotune.tune("w2", run, space=SPACE, cache_path=path)   # another workload
    assert not cached and len(calls) > n
