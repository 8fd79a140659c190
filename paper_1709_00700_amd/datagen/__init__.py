"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

This module draws random columns (``gen.c``) and writes neutral query
descriptions (plain dicts, see ``spec`` below). It contains none of the
pipeline's arithmetic: no predicate evaluation, join, hashing or aggregation.
Both sides of every parity check receive exactly the arrays produced here.

Query description ("spec"), consumed by ``oracle`` and by the library binding:

    {"builds": [{"table": str, "filters": [(col, lo, hi), ...],
                 "key": col, "payload": col}, ...],          # HASH_PUT pipelines
     "main": {"table": str,
              "filters": [(col, lo, hi), ...],                # lo <= col <= hi, conjunctive
              "cross": str, "cross_filters": [(col, lo, hi), ...],  # optional CROSS_JOIN, then FILTERs
              "probes": [(fk_col, build_index, payload_name), ...],
              "arith": [(out_name, "add"|"sub"|"mul", x, y), ...],  # x, y: attr name or int
              "project": [attr, ...],                         # projection pipeline, or
              "group_by": [attr, ...], "aggs": [(fn, attr|None, wide), ...],
              "groups_hint": int}}

Workload shapes stand in for the paper's benchmark pipelines (Section 9.2):
C1 projection (Projection Query 1/2 shape), C2 grouped aggregation
(Aggregation Query 1/2 shape), C3 star join + grouping (SSB Q4.1 shape), C4
wide scan-aggregate (TPC-H Q1 shape). The recipes are synthetic; no benchmark
data, generator or query text is reproduced.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

MASTER_SEED = 20170903
_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libhawkgen.so")
_lib = None

I64_MIN = -(1 << 63)
I64_MAX = (1 << 63) - 1


def build(force: bool = True) -> str:
    """Compile gen.c into libhawkgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", _SO + ".tmp",
               os.path.join(_HERE, "gen.c"), "-lm"]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        i64, u64, i32, u32, p = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p
        for nm in ("hg_uniform_i8", "hg_uniform_i32", "hg_uniform_i64"):
            getattr(L, nm).argtypes = [u64, u64, i64, i64, i64, i64, p]
            getattr(L, nm).restype = None
        L.hg_categorical_i8.argtypes = [u64, u64, i64, i64, p, i32, p]
        L.hg_sparse_keys_i32.argtypes = [u64, u64, i64, i64, p]
        L.hg_foreign_keys_i32.argtypes = [u64, u64, u64, i64, i64, i64, p]
        L.hg_zipf_i32.argtypes = [u64, u64, i64, i64, i64, ctypes.c_double, i32, p]
        L.hg_unit_f64.argtypes = [u64, u64, i64, i64, p]
        L.hg_splitmix64.argtypes = [u64]
        L.hg_splitmix64.restype = u64
        L.hg_draw.argtypes = [u64, u64, u64]
        L.hg_draw.restype = u64
        L.hg_scramble32.argtypes = [u32, u32]
        L.hg_scramble32.restype = u32
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


# ---------------------------------------------------------------- primitives
def uniform(seed, stream, n, lo, hi, dtype, offset=0):
    """n integers uniform in [lo, hi) of the given numpy dtype (int8/int32/int64)."""
    dt = np.dtype(dtype)
    out = np.empty(int(n), dtype=dt)
    fn = {1: "hg_uniform_i8", 4: "hg_uniform_i32", 8: "hg_uniform_i64"}[dt.itemsize]
    getattr(lib(), fn)(seed, stream, int(offset), int(n), int(lo), int(hi), _ptr(out))
    return out


def categorical_i8(seed, stream, n, probs, offset=0):
    p = np.ascontiguousarray(probs, dtype=np.float64)
    out = np.empty(int(n), dtype=np.int8)
    lib().hg_categorical_i8(seed, stream, int(offset), int(n), _ptr(p), len(p), _ptr(out))
    return out


def sparse_keys(seed, stream, n, first=0):
    out = np.empty(int(n), dtype=np.int32)
    lib().hg_sparse_keys_i32(seed, stream, int(first), int(n), _ptr(out))
    return out


def foreign_keys(seed, stream, key_stream, n, ndim, offset=0):
    out = np.empty(int(n), dtype=np.int32)
    lib().hg_foreign_keys_i32(seed, stream, key_stream, int(offset), int(n), int(ndim), _ptr(out))
    return out


def zipf(seed, stream, n, nranks, s, scramble=True, offset=0):
    out = np.empty(int(n), dtype=np.int32)
    lib().hg_zipf_i32(seed, stream, int(offset), int(n), int(nranks), float(s), int(scramble), _ptr(out))
    return out


def unit_f64(seed, stream, n, offset=0):
    out = np.empty(int(n), dtype=np.float64)
    lib().hg_unit_f64(seed, stream, int(offset), int(n), _ptr(out))
    return out


# ---------------------------------------------------------------- workloads
# full sizes of the five workload configurations
FULL_ROWS = {"c1": 1_000_000, "c2": 64 << 20, "c3": 120_000_000, "c4": 600_000_000}
C3_DIMS = (2_500, 200_000, 30_000, 80_000)
C3_DIM_SEL = (20, 5, 20, 1)      # percent of each dimension kept by its filter


def _stream(config: int, col: int) -> int:
    return (config << 16) | col


def c1_projection(n=FULL_ROWS["c1"], seed=MASTER_SEED, lo=0, hi=1000):
    """Selection + order-preserving projection: a<100 AND 200<=b<700, out c*d+a."""
    t = {k: uniform(seed, _stream(1, j), n, lo, hi, np.int32) for j, k in enumerate("abcd")}
    spec = {"builds": [],
            "main": {"table": "t",
                     "filters": [("a", I64_MIN, 99), ("b", 200, 699)],
                     "probes": [],
                     "arith": [("cd", "mul", "c", "d"), ("out", "add", "cd", "a")],
                     "project": ["out"]}}
    return {"t": t}, spec


def c2_aggregation(n=FULL_ROWS["c2"], seed=MASTER_SEED, dist="uniform", groups=16,
                   nranks=1_000_000, zipf_s=1.1, vlo=0, vhi=1_000_000):
    """Grouped COUNT/SUM/MIN/MAX of an int64 value by an int32 key.

    dist="uniform": `groups` distinct sparse keys, uniformly drawn.
    dist="zipf": ranks 1..nranks with P(r) ~ r^-zipf_s, scrambled to sparse keys.
    """
    if dist == "uniform":
        ranks = uniform(seed, _stream(2, 0), n, 0, groups, np.int32)
        k = lib().hg_scramble32
        key_of = np.array([k(r, 0x9E37) for r in range(groups)], dtype=np.uint32).view(np.int32)
        key = key_of[ranks]
        hint = groups
    elif dist == "zipf":
        key = zipf(seed, _stream(2, 1), n, nranks, zipf_s)
        hint = nranks
    else:
        raise ValueError(dist)
    v = uniform(seed, _stream(2, 2), n, vlo, vhi, np.int64)
    spec = {"builds": [],
            "main": {"table": "t", "filters": [], "probes": [], "arith": [],
                     "group_by": ["k"],
                     "aggs": [("count", None, False), ("sum", "v", False),
                              ("min", "v", False), ("max", "v", False)],
                     "groups_hint": int(hint)}}
    return {"t": {"k": key, "v": v}}, spec


def c3_star_join(n=FULL_ROWS["c3"], seed=MASTER_SEED, dims=C3_DIMS, sel=C3_DIM_SEL):
    """Four filtered dimension builds, fused probe chain, SUM(revenue) by (d0.g, d2.g)."""
    tables = {}
    builds = []
    ngroups = (7, 50, 250, 25)
    for j, nd in enumerate(dims):
        ks = _stream(3, 16 + j)
        tables[f"d{j}"] = {
            "key": sparse_keys(seed, ks, nd),
            "f": uniform(seed, _stream(3, 32 + j), nd, 0, 100, np.int32),
            "g": uniform(seed, _stream(3, 48 + j), nd, 0, ngroups[j], np.int32),
        }
        builds.append({"table": f"d{j}", "filters": [("f", 0, sel[j] - 1)],
                       "key": "key", "payload": "g"})
    fact = {f"fk{j}": foreign_keys(seed, _stream(3, j), _stream(3, 16 + j), n, nd)
            for j, nd in enumerate(dims)}
    fact["rev"] = uniform(seed, _stream(3, 8), n, 0, 1_000_000, np.int64)
    tables["f"] = fact
    spec = {"builds": builds,
            "main": {"table": "f", "filters": [],
                     "probes": [(f"fk{j}", j, f"p{j}") for j in range(len(dims))],
                     "arith": [],
                     "group_by": ["p0", "p2"],
                     "aggs": [("sum", "rev", False)],
                     "groups_hint": ngroups[0] * ngroups[2]}}
    return tables, spec


def c4_wide(n=FULL_ROWS["c4"], seed=MASTER_SEED, price_hi=100_001):
    """Wide scan-aggregate: 6 skewed groups, 8 aggregates, one exact 128-bit sum."""
    t = {
        "flag1": categorical_i8(seed, _stream(4, 0), n, [0.49, 0.49, 0.02]),
        "flag2": uniform(seed, _stream(4, 1), n, 0, 2, np.int8),
        "qty": uniform(seed, _stream(4, 2), n, 1, 51, np.int32),
        "price": uniform(seed, _stream(4, 3), n, 900, price_hi, np.int64),
        "disc": uniform(seed, _stream(4, 4), n, 0, 11, np.int32),
        "tax": uniform(seed, _stream(4, 5), n, 0, 11, np.int32),
    }
    spec = {"builds": [],
            "main": {"table": "t", "filters": [], "probes": [],
                     "arith": [("one_minus_disc", "sub", 100, "disc"),
                               ("disc_price", "mul", "price", "one_minus_disc"),
                               ("one_plus_tax", "add", 100, "tax"),
                               ("charge", "mul", "disc_price", "one_plus_tax")],
                     "group_by": ["flag1", "flag2"],
                     "aggs": [("count", None, False), ("sum", "qty", False),
                              ("sum", "price", False), ("sum", "disc_price", False),
                              ("sum", "charge", True), ("min", "price", False),
                              ("max", "disc", False), ("avg", "qty", False)],
                     "groups_hint": 6}}
    return {"t": t}, spec


def cross_join(n=20_000, m=64, nd=40, seed=MASTER_SEED, sink="project"):
    """A pipeline with a CROSS_JOIN (Table 1): rows of `t` that pass a filter,
    paired with every row of the small table `u`, a band filter on the pair
    (u.b within range, t.a again), a probe keyed by u.fk into dimension `d`,
    arithmetic over both sides; sink "project" (ab, vw, p) or "group" (COUNT,
    wide SUM, MIN, MAX, AVG by (p, b))."""
    keys = sparse_keys(seed, _stream(6, 0), nd)
    tables = {
        "d": {"key": keys, "g": uniform(seed, _stream(6, 1), nd, -3, 4, np.int32)},
        "t": {"a": uniform(seed, _stream(6, 2), n, -1000, 1000, np.int32),
              "v": uniform(seed, _stream(6, 3), n, -(1 << 40), 1 << 40, np.int64)},
        "u": {"b": uniform(seed, _stream(6, 4), m, -1000, 1000, np.int32),
              "fk": foreign_keys(seed, _stream(6, 5), _stream(6, 0), m, nd),
              "w": uniform(seed, _stream(6, 6), m, -5, 6, np.int8)},
    }
    main = {"table": "t", "filters": [("a", -800, 900)], "cross": "u",
            "cross_filters": [("b", -600, 700), ("a", -700, 900)],
            "probes": [("fk", 0, "p")], "arith": [("vw", "mul", "v", "w"), ("ab", "sub", "a", "b")]}
    if sink == "project":
        main["project"] = ["ab", "vw", "p"]
    else:
        main.update(group_by=["p", "b"], groups_hint=7 * m,
                    aggs=[("count", None, False), ("sum", "vw", True), ("min", "ab", False),
                          ("max", "v", False), ("avg", "vw", False)])
    return tables, {"builds": [{"table": "d", "filters": [], "key": "key", "payload": "g"}], "main": main}


def workload(name: str, **kw):
    """(tables, spec) for a named workload: c1, c2u (16 uniform groups), c2z (zipf), c3, c4."""
    if name == "c1":
        return c1_projection(**kw)
    if name == "c2u":
        return c2_aggregation(dist="uniform", **kw)
    if name == "c2z":
        return c2_aggregation(dist="zipf", **kw)
    if name == "c3":
        return c3_star_join(**kw)
    if name == "c4":
        return c4_wide(**kw)
    raise ValueError(name)


# ---------------------------------------------------------------- C5: mixed workload of many pipelines
# key cardinalities available in the grouping pool (groups are snapped to the nearest level)
C5_GROUP_LEVELS = (1, 16, 256, 4096, 65536, 1 << 20, 4_000_000)


def c5_pools(pool_rows, seed=MASTER_SEED + 5):
    """Shared column pools; every C5 pipeline scans a window of one of them.

    kind 1 (projection): a, b, c, d int32 uniform [0, 10^6)
    kind 2 (aggregation): f int32 uniform [0, 10^6) (selectivity filter),
        k<i> int32 keys uniform over C5_GROUP_LEVELS[i] sparse values, v int64 [0, 10^6)
    kind 3 (star join): fact fk0..fk3 into four dimensions of 2.5k/200k/30k/80k rows,
        rev int64 [0, 10^6); dims carry key, f (uniform [0, 10^6)) and g
    """
    n = int(pool_rows)
    p1 = {c: uniform(seed, _stream(5, j), n, 0, 1_000_000, np.int32) for j, c in enumerate("abcd")}
    p2 = {"f": uniform(seed, _stream(5, 8), n, 0, 1_000_000, np.int32),
          "v": uniform(seed, _stream(5, 9), n, 0, 1_000_000, np.int64)}
    sc = lib().hg_scramble32
    for i, g in enumerate(C5_GROUP_LEVELS):
        ranks = uniform(seed, _stream(5, 16 + i), n, 0, g, np.int32)
        if g <= 1 << 16:
            key_of = np.array([sc(r, 0x51 + i) for r in range(g)], dtype=np.uint32).view(np.int32)
            p2[f"k{i}"] = key_of[ranks]
        else:
            p2[f"k{i}"] = ranks   # dense keys for the large levels
    dims = {}
    ngroups = (7, 50, 250, 25)
    for j, nd in enumerate(C3_DIMS):
        dims[f"d{j}"] = {"key": sparse_keys(seed, _stream(5, 32 + j), nd),
                         "f": uniform(seed, _stream(5, 40 + j), nd, 0, 1_000_000, np.int32),
                         "g": uniform(seed, _stream(5, 48 + j), nd, 0, ngroups[j], np.int32)}
    p3 = {f"fk{j}": foreign_keys(seed, _stream(5, 56 + j), _stream(5, 32 + j), n, nd) for j, nd in enumerate(C3_DIMS)}
    p3["rev"] = uniform(seed, _stream(5, 60), n, 0, 1_000_000, np.int64)
    return {"p1": p1, "p2": p2, "p3": p3, **dims}


def c5_queries(nq=256, pool_rows=200_000_000, seed=MASTER_SEED + 5, min_rows=1_000_000, max_rows=200_000_000):
    """Seeded list of C5 pipelines: dicts with kind, window (offset, rows), target
    selectivity, groups and the neutral spec (table names refer to windows)."""
    u = unit_f64(seed, _stream(5, 100), 8 * nq).reshape(nq, 8)
    lo, hi = np.log(min_rows), np.log(max_rows)
    mu, sigma = 0.5 * (lo + hi), (np.log(max_rows / min_rows)) / 4.0
    out = []
    for i in range(nq):
        kind = 1 + int(u[i, 0] * 3)
        # ln rows ~ N(mu, sigma) by Box-Muller, clipped to [min_rows, max_rows] and the pool
        z = np.sqrt(-2.0 * np.log(max(u[i, 1], 1e-300))) * np.cos(2 * np.pi * u[i, 2])
        rows = int(np.clip(np.exp(mu + sigma * z), min_rows, max_rows))
        rows = min(rows, int(pool_rows))
        sel = float(np.exp(np.log(1e-3) + u[i, 3] * (np.log(0.5) - np.log(1e-3))))
        groups_t = float(np.exp(u[i, 4] * np.log(4e6)))
        level = int(np.argmin([abs(np.log(max(groups_t, 1)) - np.log(g)) for g in C5_GROUP_LEVELS]))
        off = int(u[i, 5] * (int(pool_rows) - rows + 1))
        thr = int(round(sel * 1_000_000)) - 1
        win = f"w{i}"
        if kind == 1:
            spec = {"builds": [], "main": {"table": win, "filters": [("a", 0, thr)], "probes": [],
                                           "arith": [("cd", "mul", "c", "d"), ("out", "add", "cd", "b")],
                                           "project": ["out"]}}
            pool = "p1"
        elif kind == 2:
            spec = {"builds": [], "main": {"table": win, "filters": [("f", 0, thr)], "probes": [], "arith": [],
                                           "group_by": [f"k{level}"] if C5_GROUP_LEVELS[level] > 1 else [],
                                           "aggs": [("count", None, False), ("sum", "v", False),
                                                    ("min", "v", False), ("max", "v", False)],
                                           "groups_hint": int(C5_GROUP_LEVELS[level])}}
            pool = "p2"
        else:
            # four dimension filters whose product is about the target selectivity
            per = sel ** 0.25
            dthr = int(round(per * 1_000_000)) - 1
            spec = {"builds": [{"table": f"d{j}", "filters": [("f", 0, dthr)], "key": "key", "payload": "g"}
                               for j in range(4)],
                    "main": {"table": win, "filters": [], "probes": [(f"fk{j}", j, f"p{j}") for j in range(4)],
                             "arith": [], "group_by": ["p0", "p2"], "aggs": [("sum", "rev", False)],
                             "groups_hint": 7 * 250}}
            pool = "p3"
        out.append({"kind": kind, "pool": pool, "offset": off, "rows": rows, "selectivity": sel,
                    "groups": int(C5_GROUP_LEVELS[level]) if kind == 2 else (1750 if kind == 3 else 0),
                    "window": win, "spec": spec})
    return out


def c5_window_tables(pools, q):
    """numpy views of the tables a C5 pipeline reads (its window, plus dimensions)."""
    pool = pools[q["pool"]]
    t = {q["window"]: {c: a[q["offset"]:q["offset"] + q["rows"]] for c, a in pool.items()}}
    for b in q["spec"]["builds"]:
        t[b["table"]] = pools[b["table"]]
    return t
