"""Host logic of the pick-quality evaluation (no GPU): the ratios of each
picker's and Algorithm 1's runtimes to every query's exhaustive best, on
stubbed timings whose ratios are known by hand."""
import math

import pytest

from paper_1709_00700_amd import optimizer


class _Query:
    def __init__(self, kind):
        self.kind = kind


class _Picker:
    def __init__(self, picks):
        self.picks = picks

    def pick(self, queries):
        return self.picks, None


def test_pick_quality_ratios(monkeypatch):
    qs = [_Query(1), _Query(2)]
    # exhaustive timings per query: variant key -> ms
    tables = [{"a": 1.0, "b": 2.0, "c": 8.0}, {"a": 4.0, "b": 1.0, "c": 2.0}]
    monkeypatch.setattr(optimizer, "exhaustive", lambda ctx, q, reps, lim, **kw: dict(tables[qs.index(q)]))
    monkeypatch.setattr(optimizer, "variant_key", lambda q, v, tabled=None: v)
    alg1 = {1: ("c", None), 2: ("c", None)}
    out = optimizer.pick_quality(None, qs, _Picker(["a", "a"]), reps=1, limit_ms=10.0, alg1=alg1,
                                 extra={"other": _Picker(["b", "b"])})
    assert out["queries"] == 2
    # model picks a: ratios 1 and 4
    assert out["model"]["geomean_ratio"] == pytest.approx(2.0)
    assert out["model"]["total_ratio"] == pytest.approx((1.0 + 4.0) / (1.0 + 1.0))
    assert out["model"]["max_ratio"] == pytest.approx(4.0)
    # the extra picker takes b: ratios 2 and 1
    assert out["other"]["geomean_ratio"] == pytest.approx(math.sqrt(2.0))
    assert out["other"]["total_ratio"] == pytest.approx(3.0 / 2.0)
    # Algorithm 1's one variant per kind is c: ratios 8 and 2
    assert out["alg1"]["geomean_ratio"] == pytest.approx(4.0)
    assert out["alg1"]["max_ratio"] == pytest.approx(8.0)
    rows = out["per_query"]
    assert [r["best"] for r in rows] == ["a", "b"]
    assert [r["pick"] for r in rows] == ["a", "a"] and [r["other"] for r in rows] == ["b", "b"]
    assert all(r["alg1"] == "c" for r in rows)


def test_pick_quality_pruned_pick(monkeypatch):
    # a pick outside the exhaustive table is timed on its own; a pruned one (inf) is counted, not averaged
    qs = [_Query(1), _Query(1)]
    tables = [{"a": 1.0, "b": 3.0}, {"a": 2.0, "b": 2.0}]
    monkeypatch.setattr(optimizer, "exhaustive", lambda ctx, q, reps, lim, **kw: dict(tables[qs.index(q)]))
    monkeypatch.setattr(optimizer, "variant_key", lambda q, v, tabled=None: v)
    monkeypatch.setattr(optimizer, "timed", lambda ctx, q, v, reps, lim: math.inf)
    out = optimizer.pick_quality(None, qs, _Picker(["z", "a"]), reps=1, limit_ms=10.0, alg1={1: ("b", None)})
    assert out["model"]["pruned_picks"] == 1
    assert out["model"]["geomean_ratio"] == pytest.approx(1.0)  # over the finite ratio (query 2: 2/2)
    assert out["alg1"]["pruned_picks"] == 0
    assert out["alg1"]["geomean_ratio"] == pytest.approx(math.sqrt(3.0 * 1.0))


def test_exhaustive_prunes_relative_to_the_running_best(monkeypatch):
    """With factor f, each variant after the first ones is timed under the limit
    min(limit_ms, f * fastest so far); the `first` variants get limit_ms."""
    class V:
        def __init__(self, k, ms):
            self.k, self.ms, self.ht, self.hash = k, ms, 0, 0
    space = [V("a", 5.0), V("b", 2.0), V("c", 30.0), V("d", 1.0), V("e", 9.0)]
    seen = []

    def timed(ctx, q, v, reps, lim):
        seen.append((v.k, lim))
        return v.ms if v.ms <= lim else math.inf

    monkeypatch.setattr(optimizer.hawk, "variant_space", lambda q: space)
    monkeypatch.setattr(optimizer, "variant_key", lambda q, v, tabled=None: v.k)
    monkeypatch.setattr(optimizer, "timed", timed)
    out = optimizer.exhaustive(None, None, reps=1, limit_ms=100.0, factor=4.0, first=[space[4]])
    # e first (limit 100), then a (4*9), b (4*5), c (4*2 -> pruned), d (4*2), and e is not timed again
    assert seen == [("e", 100.0), ("a", 36.0), ("b", 20.0), ("c", 8.0), ("d", 8.0)]
    assert out == {"e": 9.0, "a": 5.0, "b": 2.0, "c": math.inf, "d": 1.0}


def test_pick_quality_confirms_the_finalists(monkeypatch):
    """With confirm_reps, the search's best and the picks are timed again and
    compared on those times: a best that was only lucky in the search loses
    its place to a pick that is as fast when both are timed alike."""
    class V:
        def __init__(self, k):
            self.k, self.ht, self.hash = k, 0, 0
    space = [V("a"), V("b"), V("c")]
    qs = [_Query(2)]
    noisy = {"a": 1.0, "b": 1.2, "c": 3.0}        # the search's medians
    confirmed = {"a": 1.3, "b": 1.2, "c": 3.1}    # the finalists timed again
    retimed = []

    def timed(ctx, q, v, reps, lim):
        retimed.append((v.k, reps))
        return confirmed[v.k]

    monkeypatch.setattr(optimizer, "exhaustive", lambda ctx, q, reps, lim, **kw: dict(noisy))
    monkeypatch.setattr(optimizer.hawk, "variant_space", lambda q: space)
    monkeypatch.setattr(optimizer, "variant_key", lambda q, v, tabled=None: v.k)
    monkeypatch.setattr(optimizer, "timed", timed)
    out = optimizer.pick_quality(None, qs, _Picker([space[1]]), reps=2, limit_ms=10.0,
                                 alg1={2: (space[2], None)}, confirm_reps=5)
    # finalists: the pick b, Algorithm 1's c and the search's best a, each timed with 5 runs
    assert sorted(retimed) == [("a", 5), ("b", 5), ("c", 5)]
    row = out["per_query"][0]
    assert row["best"] == "b" and row["best_ms"] == pytest.approx(1.2)
    assert out["model"]["geomean_ratio"] == pytest.approx(1.0)
    assert out["alg1"]["geomean_ratio"] == pytest.approx(3.1 / 1.2)
