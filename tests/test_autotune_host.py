"""The autotuner's search logic on the host: a fake knob store and a fake
timer stand in for the library and the GPU."""
import json

import pytest

from paper_2303_08394_amd import autotune as A
from paper_2303_08394_amd import kifmm as K


class FakeKnobs:
    def __init__(self, start, cost):
        self.v = dict(start)
        self.cost = cost  # dict of knob settings -> ms
        self.timed = []

    def get(self, k):
        return self.v[k]

    def set_(self, k, v):
        self.v[k] = v

    def timer(self):
        self.timed.append(dict(self.v))
        return self.cost(self.v)


SPACE = (("a", (1, 2, 3)), ("b", (0, 1)))


def test_coordinate_descent_keeps_the_fastest():
    # separable cost: a = 3 and b = 1 are best
    f = FakeKnobs({"a": 1, "b": 0}, lambda v: 10.0 - 2.0 * (v["a"] == 3) - 1.0 * (v["b"] == 1))
    r = A.search(None, space=SPACE, timer=f.timer, get=f.get, set_=f.set_, confirm=0)
    assert r.best == {"a": 3, "b": 1} and f.v == r.best
    assert r.start_ms == 10.0 and r.best_ms == 7.0
    # start + 2 other values of a + 1 other value of b, b timed with a at its best
    assert len(r.trials) == 4 and f.timed[-1] == {"a": 3, "b": 1}
    # with confirmation: start and best timed 3 more times each, alternately
    f.v = {"a": 1, "b": 0}
    r = A.search(None, space=SPACE, timer=f.timer, get=f.get, set_=f.set_, confirm=3)
    assert r.best == {"a": 3, "b": 1} and f.v == r.best and r.best_ms == 7.0
    assert len(r.trials) == 10
    assert [t[0] for t in r.trials[4:]] == [{"a": 1, "b": 0}, {"a": 3, "b": 1}] * 3


def test_a_lucky_timing_is_not_kept():
    """A candidate that timed fast once but not on re-timing is dropped and
    the starting layout is put back."""
    calls = {"n": 0}

    def cost(v):
        calls["n"] += 1
        return 8.0 if (v["a"] == 2 and calls["n"] == 2) else 10.0

    f = FakeKnobs({"a": 1, "b": 0}, cost)
    r = A.search(None, space=SPACE, timer=f.timer, get=f.get, set_=f.set_, confirm=3)
    assert r.best == {"a": 1, "b": 0} and f.v == r.best and r.best_ms == 10.0


def test_small_gains_do_not_move_the_layout():
    f = FakeKnobs({"a": 1, "b": 0}, lambda v: 10.0 - 0.05 * (v["a"] == 2))  # 0.5% faster
    r = A.search(None, space=SPACE, timer=f.timer, get=f.get, set_=f.set_, min_gain=0.01)
    assert r.best == {"a": 1, "b": 0} and f.v == r.best
    r = A.search(None, space=SPACE, timer=f.timer, get=f.get, set_=f.set_, min_gain=0.001)
    assert r.best["a"] == 2


def test_a_failing_trial_restores_its_knob():
    def cost(v):
        if v["b"] == 1:
            raise RuntimeError("trial failed")
        return 5.0

    f = FakeKnobs({"a": 1, "b": 0}, lambda v: cost(v) - (v["a"] == 3))
    with pytest.raises(RuntimeError):
        A.search(None, space=SPACE, timer=f.timer, get=f.get, set_=f.set_)
    assert f.v == {"a": 1, "b": 0}  # the starting layout, though a = 3 had been kept


def test_search_needs_a_stream_or_a_timer():
    with pytest.raises(ValueError):
        A.search(lambda: None, None, space=SPACE, get=lambda k: 1, set_=lambda k, v: None)


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    f = FakeKnobs({"a": 1, "b": 0}, lambda v: 9.0 - (v["a"] == 2))
    r = A.autotune(None, None, key="w1", cache_path=path, space=SPACE, timer=f.timer, get=f.get, set_=f.set_)
    assert not r.from_cache and r.best == {"a": 2, "b": 0}
    assert json.load(open(path)) == {"w1": {"a": 2, "b": 0}}

    def no_timing():
        raise AssertionError("a cached layout is applied without timing")

    g = FakeKnobs({"a": 1, "b": 1}, None)
    r2 = A.autotune(None, None, key="w1", cache_path=path, space=SPACE, timer=no_timing, get=g.get, set_=g.set_)
    assert r2.from_cache and g.v == {"a": 2, "b": 0}
    # another workload is searched and added beside the first
    r3 = A.autotune(None, None, key="w2", cache_path=path, space=SPACE, timer=f.timer, get=f.get, set_=f.set_)
    assert not r3.from_cache and set(json.load(open(path))) == {"w1", "w2"}


def test_space_is_valid_for_the_library():
    """Every candidate is a value kifmm_set_tuning accepts; the first of each
    knob is its default, which kifmm_get_tuning reports."""
    for k, cands in A.SPACE:
        assert K.get_tuning(k) == cands[0]
    try:
        for k, cands in A.SPACE:
            for v in cands:
                K.set_tuning(k, v)
                assert K.get_tuning(k) == v
    finally:
        for k, cands in A.SPACE:
            K.set_tuning(k, cands[0])
    with pytest.raises(K.KifmmError, match="unknown"):
        K.get_tuning("no_such_key")


def test_signature_names_the_workload():
    """The cache key separates workloads by tree shape, order, precision and
    right-hand sides (host only: no device is needed to form it)."""
    import numpy as np

    x = np.random.default_rng(0).random((2000, 3))
    t1 = K.Tree(x, uniform_depth=2, center=(0.5, 0.5, 0.5), halfwidth=0.5)
    t2 = K.Tree(x, ncrit=32, max_depth=8, center=(0.5, 0.5, 0.5), halfwidth=0.5)
    o4 = K.Operators(4)
    o5 = K.Operators(5)
    keys = {A.signature(t1, o4, "fp32"), A.signature(t2, o4, "fp32"), A.signature(t1, o5, "fp32"),
            A.signature(t1, o4, "bf16x3"), A.signature(t1, o4, "fp32", n_rhs=4),
            A.signature(t1, o4, "fp32", what="batch")}
    assert len(keys) == 6
    assert A.signature(t1, o4, "fp32") == A.signature(t1, o4, "fp32")
