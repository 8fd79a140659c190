"""Pins of the CPU oracle to things other than itself (no GPU needed).

* hand-worked examples (tests/golden/, each citing the passage it follows);
* row-at-a-time brute force with nested-loop joins and per-group rescans on
  tiny random tables (tests/bruteforce.py);
* invariants and closed forms at medium sizes, checked with independent numpy
  reductions (group counts sum to the selected rows, per-group sums add up to
  the total, join cardinality, MIN <= MAX, arithmetic-series sums);
* exact 128-bit sums against Python integers on an overflow-forcing input;
* AVG within 1e-12 relative of the exact rational.
"""
import glob
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import bruteforce
import oracle
from paper_1709_00700_amd import datagen as dg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1


def load_golden(path):
    with open(path) as f:
        g = json.load(f)
    tables = {t: {c: np.array(v["values"], dtype=v["dtype"]) for c, v in cols.items()}
              for t, cols in g["tables"].items()}
    spec = g["spec"]
    spec["main"]["filters"] = [tuple(x) for x in spec["main"].get("filters", [])]
    spec["main"]["probes"] = [tuple(x) for x in spec["main"].get("probes", [])]
    spec["main"]["arith"] = [tuple(x) for x in spec["main"].get("arith", [])]
    if "aggs" in spec["main"]:
        spec["main"]["aggs"] = [tuple(x) for x in spec["main"]["aggs"]]
    for b in spec["builds"]:
        b["filters"] = [tuple(x) for x in b.get("filters", [])]
    return tables, spec, g["expected"], g["citation"]


def as_py(res):
    """Oracle result -> plain Python lists (wide sums as int, AVG as float)."""
    if res["kind"] == "project":
        return {"kind": "project", "rows": res["rows"], "cols": [list(map(int, c)) for c in res["cols"]]}
    out = {"kind": "aggregate", "rows": res["rows"], "keys": [list(map(int, k)) for k in res["keys"]],
           "count": list(map(int, res["count"])), "aggs": []}
    for a in res["aggs"]:
        out["aggs"].append([float(x) if isinstance(x, (float, np.floating)) else int(x) for x in a])
    return out


def assert_matches_bruteforce(res, bf, spec):
    r = as_py(res)
    assert r["rows"] == bf["rows"]
    if r["kind"] == "project":
        assert r["cols"] == bf["cols"]
        return
    assert r["keys"] == bf["keys"]
    assert r["count"] == bf["count"]
    for j, (fn, _, _) in enumerate(spec["main"]["aggs"]):
        if fn == "avg":
            for got, exact in zip(r["aggs"][j], bf["aggs"][j]):
                if exact is None:
                    assert got != got  # NaN for an empty AGGREGATE
                else:
                    assert abs(Fraction(got) - exact) <= Fraction(1, 10**12) * abs(exact)
        else:
            assert r["aggs"][j] == bf["aggs"][j], (fn, j)


# ------------------------------------------------------------------ golden
@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLDEN, "*.json"))),
                         ids=lambda p: os.path.basename(p))
def test_golden(path):
    tables, spec, exp, cite = load_golden(path)
    assert cite
    r = as_py(oracle.run(tables, spec))
    assert r["rows"] == exp["rows"]
    if exp["kind"] == "project":
        assert r["cols"] == exp["cols"]
    else:
        assert r["keys"] == exp["keys"]
        assert r["count"] == exp["count"]
        for j, (fn, _, _) in enumerate(spec["main"]["aggs"]):
            if fn == "avg":
                for got, (num, den) in zip(r["aggs"][j], exp["aggs"][j]):
                    assert abs(Fraction(got) - Fraction(num, den)) <= Fraction(1, 10**12) * abs(Fraction(num, den))
            else:
                assert r["aggs"][j] == exp["aggs"][j]
    # the brute force agrees with the hand-worked values too
    bf = bruteforce.run(tables, spec)
    assert_matches_bruteforce(oracle.run(tables, spec), bf, spec)


# ------------------------------------------------------------------ brute force, tiny random tables
def _rand_table(rng, n, spec_cols):
    return {c: rng.integers(lo, hi, size=n, endpoint=True).astype(dt) for c, (dt, lo, hi) in spec_cols.items()}


@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_projection(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(0, 300))
    t = _rand_table(rng, n, {"a": (np.int32, -20, 20), "b": (np.int8, -128, 127),
                             "c": (np.int64, -(1 << 40), 1 << 40), "d": (np.int32, -(1 << 31), (1 << 31) - 1)})
    spec = {"builds": [], "main": {"table": "t",
                                   "filters": [("a", -5, 10), ("b", int(rng.integers(-128, 0)), 127)],
                                   "probes": [],
                                   "arith": [("cd", "mul", "c", "d"), ("x", "sub", "cd", "a"),
                                             ("y", "sub", 3, "b"), ("z", "add", "y", "x")],
                                   "project": ["z", "a", "cd"]}}
    assert_matches_bruteforce(oracle.run({"t": t}, spec), bruteforce.run({"t": t}, spec), spec)


@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_join_group(seed):
    rng = np.random.default_rng(100 + seed)
    nd = [int(rng.integers(1, 30)) for _ in range(3)]
    tables = {}
    builds = []
    for j, k in enumerate(nd):
        keys = rng.choice(np.arange(-50, 50), size=k, replace=False).astype(np.int32)
        tables[f"d{j}"] = {"key": keys, "f": rng.integers(0, 10, size=k).astype(np.int32),
                           "g": rng.integers(-3, 4, size=k).astype(np.int32)}
        builds.append({"table": f"d{j}", "filters": [("f", 0, int(rng.integers(0, 10)))],
                       "key": "key", "payload": "g"})
    n = int(rng.integers(0, 250))
    tables["f"] = {f"fk{j}": rng.integers(-50, 50, size=n).astype(np.int32) for j in range(3)}
    tables["f"]["v"] = rng.integers(-(1 << 62), 1 << 62, size=n).astype(np.int64)
    tables["f"]["w"] = rng.integers(-4, 5, size=n).astype(np.int8)
    spec = {"builds": builds,
            "main": {"table": "f", "filters": [("w", -3, 4)],
                     "probes": [("fk0", 0, "p0"), ("fk1", 1, "p1"), ("fk2", 2, "p2")],
                     "arith": [("vw", "mul", "v", "w")],
                     "group_by": ["p0", "p2"] if seed % 3 else (["w"] if seed % 2 else []),
                     "aggs": [("count", None, False), ("sum", "v", True), ("sum", "vw", False),
                              ("min", "v", False), ("max", "p1", False), ("avg", "v", False),
                              ("sum", "vw", True)],
                     "groups_hint": 64}}
    assert_matches_bruteforce(oracle.run(tables, spec), bruteforce.run(tables, spec), spec)


def cross_case(rng, n, ni, nd):
    """A pipeline with a CROSS_JOIN (Table 1) over random tiny tables: a
    filter on the looped table, the cross product with table `u`, a filter
    on either side, a probe keyed by a column of `u`, arithmetic over both."""
    keys = rng.choice(np.arange(-20, 20), size=nd, replace=False).astype(np.int32)
    tables = {"d": {"key": keys, "g": rng.integers(-3, 4, size=nd).astype(np.int32)},
              "t": {"a": rng.integers(-10, 10, size=n).astype(np.int32),
                    "v": rng.integers(-(1 << 40), 1 << 40, size=n).astype(np.int64)},
              "u": {"b": rng.integers(-10, 10, size=ni).astype(np.int32),
                    "fk": rng.integers(-20, 20, size=ni).astype(np.int32),
                    "w": rng.integers(-5, 6, size=ni).astype(np.int8)}}
    main = {"table": "t", "filters": [("a", -6, 9)], "cross": "u", "cross_filters": [("b", -4, 8), ("a", -5, 9)],
            "probes": [("fk", 0, "p")], "arith": [("vw", "mul", "v", "w"), ("ab", "sub", "a", "b")]}
    return tables, {"builds": [{"table": "d", "filters": [], "key": "key", "payload": "g"}], "main": main}


@pytest.mark.parametrize("seed", range(8))
def test_bruteforce_cross_join(seed):
    """CROSS_JOIN against nested loops: projection in (row, second-table
    row) order, and grouping over attributes of both sides and a payload."""
    rng = np.random.default_rng(300 + seed)
    tables, spec = cross_case(rng, int(rng.integers(0, 40)), int(rng.integers(0, 25)), int(rng.integers(1, 20)))
    proj = {**spec, "main": {**spec["main"], "project": ["ab", "vw", "p", "fk"]}}
    assert_matches_bruteforce(oracle.run(tables, proj), bruteforce.run(tables, proj), proj)
    grp = {**spec, "main": {**spec["main"], "group_by": ["p", "b"],
                            "aggs": [("count", None, False), ("sum", "vw", True), ("min", "ab", False),
                                     ("max", "v", False), ("avg", "vw", False)], "groups_hint": 64}}
    assert_matches_bruteforce(oracle.run(tables, grp), bruteforce.run(tables, grp), grp)


def test_cross_join_closed_forms():
    """Without filters a CROSS_JOIN of n and m rows has n*m tuples in
    row-major order, and SUM over an attribute of one side is its column sum
    times the other side's row count."""
    n, m = 37, 11
    t = {"x": np.arange(n, dtype=np.int64) * 3 - 50}
    u = {"y": np.arange(m, dtype=np.int32) - 4}
    spec = {"builds": [], "main": {"table": "t", "filters": [], "cross": "u", "probes": [], "arith": [],
                                   "project": ["x", "y"]}}
    r = oracle.run({"t": t, "u": u}, spec)
    assert r["rows"] == n * m
    assert np.array_equal(r["cols"][0], np.repeat(t["x"], m))
    assert np.array_equal(r["cols"][1], np.tile(u["y"].astype(np.int64), n))
    agg = {"builds": [], "main": {"table": "t", "filters": [], "cross": "u", "probes": [], "arith": [],
                                  "aggs": [("count", None, False), ("sum", "x", False), ("sum", "y", False)]}}
    r = oracle.run({"t": t, "u": u}, agg)
    assert int(r["count"][0]) == n * m
    assert int(r["aggs"][1][0]) == int(t["x"].sum()) * m
    assert int(r["aggs"][2][0]) == int(u["y"].sum()) * n
    # an empty side empties the product
    r = oracle.run({"t": t, "u": {"y": u["y"][:0]}}, spec)
    assert r["rows"] == 0


def test_duplicate_build_key_is_error():
    tables = {"d": {"key": np.array([1, 2, 1], np.int32), "g": np.array([0, 1, 2], np.int32)},
              "f": {"fk": np.array([1, 2], np.int32)}}
    spec = {"builds": [{"table": "d", "filters": [], "key": "key", "payload": "g"}],
            "main": {"table": "f", "filters": [], "probes": [("fk", 0, "p")], "arith": [], "project": ["p"]}}
    with pytest.raises(oracle.OracleError) as e:
        oracle.run(tables, spec)
    assert e.value.code == oracle.ORC_E_DUPKEY
    assert bruteforce.run(tables, spec) == {"error": "dupkey"}
    # filtering the duplicate away makes the build legal
    tables["d"]["f"] = np.array([0, 0, 1], np.int32)
    spec["builds"][0]["filters"] = [("f", 0, 0)]
    assert oracle.run(tables, spec)["cols"][0].tolist() == [0, 1]


def test_sentinel_like_keys():
    """Keys equal to all-ones/extreme words are ordinary keys for the definition."""
    keys = np.array([-1, I64_MIN >> 32, (1 << 31) - 1, -(1 << 31), 0, -1, -(1 << 31)], np.int32)
    t = {"k": keys, "k2": np.array([-1, -1, -1, -1, 0, -1, 7], np.int32), "v": np.arange(7, dtype=np.int64)}
    spec = {"builds": [], "main": {"table": "t", "filters": [], "probes": [], "arith": [],
                                   "group_by": ["k", "k2"],
                                   "aggs": [("count", None, False), ("sum", "v", False)], "groups_hint": 8}}
    assert_matches_bruteforce(oracle.run({"t": t}, spec), bruteforce.run({"t": t}, spec), spec)


def test_empty_inputs():
    t = {"a": np.zeros(0, np.int32), "v": np.zeros(0, np.int64)}
    sp = {"builds": [], "main": {"table": "t", "filters": [("a", 0, 5)], "probes": [], "arith": [],
                                 "project": ["v"]}}
    assert oracle.run({"t": t}, sp)["rows"] == 0
    sg = {"builds": [], "main": {"table": "t", "filters": [], "probes": [], "arith": [],
                                 "group_by": ["a"], "aggs": [("sum", "v", False)], "groups_hint": 1}}
    assert oracle.run({"t": t}, sg)["rows"] == 0
    # AGGREGATE without groups: one row with the identities
    sa = {"builds": [], "main": {"table": "t", "filters": [], "probes": [], "arith": [], "group_by": [],
                                 "aggs": [("count", None, False), ("sum", "v", False), ("min", "v", False),
                                          ("max", "v", False), ("avg", "v", False)], "groups_hint": 1}}
    r = oracle.run({"t": t}, sa)
    assert r["rows"] == 1 and r["count"].tolist() == [0]
    assert [int(a[0]) for a in r["aggs"][:4]] == [0, 0, I64_MAX, I64_MIN]
    assert np.isnan(r["aggs"][4][0])


# ------------------------------------------------------------------ invariants at medium size
def test_c1_invariants():
    tables, spec = dg.c1_projection(n=300_000)
    t = tables["t"]
    r = oracle.run(tables, spec)
    mask = (t["a"] < 100) & (t["b"] >= 200) & (t["b"] < 700)
    assert r["rows"] == int(mask.sum())
    exp = t["c"][mask].astype(np.int64) * t["d"][mask].astype(np.int64) + t["a"][mask]
    np.testing.assert_array_equal(r["cols"][0], exp)
    # selectivity is about 5 % by construction
    assert 0.045 < r["rows"] / 300_000 < 0.055


def test_c1_closed_form():
    """a_i = i mod 1000, b_i = (7 i) mod 1000 over 1000 k rows: counts are exact."""
    k = 37
    i = np.arange(1000 * k, dtype=np.int64)
    t = {"a": (i % 1000).astype(np.int32), "b": ((7 * i) % 1000).astype(np.int32),
         "c": np.ones_like(i, dtype=np.int32), "d": (i % 3).astype(np.int32)}
    _, spec = dg.c1_projection(n=1)
    r = oracle.run({"t": t}, spec)
    # within each block of 1000 rows, a<100 picks i%1000 in [0,100); 7*i%1000 in [200,700):
    per_block = sum(1 for a in range(100) if 200 <= (7 * a) % 1000 < 700)
    assert r["rows"] == per_block * k
    # out = 1*(i%3) + i%1000 for those rows, in row order
    sel = [j for j in range(1000 * k) if j % 1000 < 100 and 200 <= (7 * j) % 1000 < 700]
    assert r["cols"][0].tolist() == [j % 3 + j % 1000 for j in sel]


@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_c2_invariants(dist):
    tables, spec = dg.c2_aggregation(n=400_000, dist=dist, nranks=50_000)
    t = tables["t"]
    r = oracle.run(tables, spec)
    cnt, s, mn, mx = r["aggs"]
    assert int(cnt.sum()) == 400_000 == int(r["count"].sum())
    assert int(s.sum()) == int(t["v"].sum())
    assert (mn <= mx).all()
    assert r["rows"] == np.unique(t["k"]).size
    keys = r["keys"][0]
    assert (np.diff(keys) > 0).all()
    # a few groups re-derived with masks
    for j in np.linspace(0, r["rows"] - 1, 7).astype(int):
        m = t["k"] == keys[j]
        assert cnt[j] == m.sum() and s[j] == t["v"][m].sum()
        assert mn[j] == t["v"][m].min() and mx[j] == t["v"][m].max()


def test_c2_closed_form_series():
    """key = i mod G, v = i: per-group count and sum are arithmetic series."""
    G, n = 16, 160_003
    i = np.arange(n, dtype=np.int64)
    t = {"k": (i % G).astype(np.int32), "v": i}
    _, spec = dg.c2_aggregation(n=1)
    r = oracle.run({"t": t}, spec)
    for g in range(G):
        c = (n - g + G - 1) // G
        assert r["count"][g] == c
        assert r["aggs"][1][g] == c * g + G * c * (c - 1) // 2
        assert r["aggs"][2][g] == g and r["aggs"][3][g] == g + G * (c - 1)


def test_c3_join_cardinality():
    tables, spec = dg.c3_star_join(n=400_000, dims=(250, 2000, 300, 800), sel=(60, 50, 60, 40))
    r = oracle.run(tables, spec)
    f = tables["f"]
    alive = np.ones(400_000, dtype=bool)
    pay = []
    for j in range(4):
        d = tables[f"d{j}"]
        keep = d["f"] <= spec["builds"][j]["filters"][0][2]
        alive &= np.isin(f[f"fk{j}"], d["key"][keep])
        order = np.argsort(d["key"])
        pos = np.searchsorted(d["key"][order], f[f"fk{j}"])
        pay.append(d["g"][order][np.minimum(pos, len(order) - 1)])
    assert int(r["count"].sum()) == int(alive.sum())
    assert int(r["aggs"][0].sum()) == int(f["rev"][alive].sum())
    grp = set(zip(pay[0][alive].tolist(), pay[2][alive].tolist()))
    assert r["rows"] == len(grp)


def test_c4_exact_wide_and_avg():
    tables, spec = dg.c4_wide(n=200_000, price_hi=1 << 40)
    t = tables["t"]
    r = oracle.run(tables, spec)
    assert r["rows"] == 6
    price = t["price"].astype(object)
    for j in range(6):
        f1, f2 = int(r["keys"][0][j]), int(r["keys"][1][j])
        m = (t["flag1"] == f1) & (t["flag2"] == f2)
        pm, dm, tm = price[m], t["disc"][m].astype(object), t["tax"][m].astype(object)
        charge = sum(p * (100 - d) * (100 + x) for p, d, x in zip(pm, dm, tm))
        assert r["aggs"][4][j] == charge                       # exact 128-bit
        assert r["aggs"][0][j] == m.sum()
        assert r["aggs"][1][j] == int(t["qty"][m].sum())
        assert r["aggs"][5][j] == t["price"][m].min() and r["aggs"][6][j] == t["disc"][m].max()
        exact_avg = Fraction(int(t["qty"][m].sum()), int(m.sum()))
        assert abs(Fraction(float(r["aggs"][7][j])) - exact_avg) <= Fraction(1, 10**12) * exact_avg
    # with prices up to 2^40 the per-group charge sum passes 2^63: only the wide sum is exact
    assert max(r["aggs"][4]) > (1 << 63)


def test_wide_sum_negative_overflow():
    rng = np.random.default_rng(7)
    n = 3000
    v = rng.integers(-(1 << 63), (1 << 63) - 1, size=n, dtype=np.int64)
    g = rng.integers(0, 3, size=n).astype(np.int8)
    spec = {"builds": [], "main": {"table": "t", "filters": [], "probes": [], "arith": [], "group_by": ["g"],
                                   "aggs": [("sum", "v", True), ("sum", "v", False)], "groups_hint": 3}}
    r = oracle.run({"t": {"g": g, "v": v}}, spec)
    for j in range(3):
        exact = sum(int(x) for x in v[g == j])
        assert r["aggs"][0][j] == exact
        assert int(r["aggs"][1][j]) == bruteforce.to_i64(exact)


# ------------------------------------------------------------------ the row-partitioned driver
def _same_answer(a, b):
    pa, pb = as_py(a), as_py(b)
    for r in (pa, pb):
        if r["kind"] == "aggregate":  # NaN != NaN: compare AVG of empty groups by their text
            r["aggs"] = [[repr(x) for x in col] for col in r["aggs"]]
    assert pa == pb


@pytest.mark.parametrize("threads", [2, 3, 7])
def test_parallel_driver_is_the_single_threaded_answer(threads):
    """The all-cores oracle splits the main pipeline's rows into contiguous
    ranges and merges their results; it must give the single-threaded answer
    (itself pinned above), including ragged range sizes, empty ranges, the
    sentinel-free AGGREGATE row and 128-bit sums and AVG."""
    cases = [dg.c1_projection(n=30_011), dg.c2_aggregation(n=40_007, dist="zipf", nranks=3000),
             dg.c3_star_join(n=20_003, dims=(50, 400, 60, 160), sel=(60, 50, 60, 40)),
             dg.c4_wide(n=25_001, price_hi=1 << 40), dg.c1_projection(n=5)]
    tables, spec = dg.c4_wide(n=9_999)
    spec["main"]["group_by"] = []
    spec["main"]["filters"] = [("qty", 10, 40)]
    cases.append((tables, spec))
    tables, spec = dg.c4_wide(n=100)
    spec["main"]["group_by"] = []
    spec["main"]["filters"] = [("qty", 100, 200)]  # nothing qualifies
    cases.append((tables, spec))
    for tables, spec in cases:
        _same_answer(oracle.run(tables, spec), oracle.run(tables, spec, threads=threads))
