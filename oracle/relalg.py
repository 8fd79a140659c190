"""Relational-plan oracle: TEST INFRASTRUCTURE ONLY.

Evaluates a relational operator tree directly, node by node, over numpy
columns, with no pipelines: it knows nothing of the produce/consume
partitioning (Section 2.1) that the library applies to the same plan, so a
plan run through the library's planner and kernels can be checked against
the plain relational answer. Only ``tests/`` may import it.

Plan format (shared with the library binding, which only marshals it):

    {"root": k, "nodes": [node, ...]} with nodes
    {"op": "scan", "table": name}
    {"op": "select", "input": i, "attr": a, "lo": lo, "hi": hi}         lo <= a <= hi
    {"op": "map", "input": i, "out": c, "fn": "add"|"sub"|"mul", "x": a|int, "y": b|int}
    {"op": "hash_join", "input": i, "build": j, "probe_key": a, "build_key": b, "payload": c}
        inner equi-join of i's tuples with j's on i.a = j.b (j's keys unique);
        the result is i's tuple plus j's attribute c
    {"op": "cross_join", "input": i, "right": j}                        every i tuple with every j tuple
    {"op": "group_by", "input": i, "keys": [...], "aggs": [(fn, attr|None, wide), ...], "groups_hint": g}
    {"op": "project", "input": i, "attrs": [...]}

The answer has the layout of ``oracle.run``: projection rows in the order of
the input (a join keeps the order of its input side, a cross join is
row-major), groups sorted by key, exact sums.
"""
from __future__ import annotations

import numpy as np

M64 = 1 << 64


class DupKey(Exception):
    """A hash join's build side holds one key twice."""


def _wrap(v: np.ndarray) -> np.ndarray:
    """64-bit two's complement of Python-integer results."""
    return np.array([((int(x) + (1 << 63)) % M64) - (1 << 63) for x in v], dtype=np.int64)


def _eval(plan: dict, k: int, tables: dict) -> dict:
    """The relation (attribute name -> int64 column) that node k yields."""
    nd = plan["nodes"][k]
    op = nd["op"]
    if op == "scan":
        return {c: np.asarray(v).astype(np.int64) for c, v in tables[nd["table"]].items()}
    if op == "select":
        r = _eval(plan, nd["input"], tables)
        keep = (r[nd["attr"]] >= nd["lo"]) & (r[nd["attr"]] <= nd["hi"])
        return {c: v[keep] for c, v in r.items()}
    if op == "map":
        r = _eval(plan, nd["input"], tables)
        n = len(next(iter(r.values())))
        x = r[nd["x"]] if isinstance(nd["x"], str) else np.full(n, nd["x"], dtype=np.int64)
        y = r[nd["y"]] if isinstance(nd["y"], str) else np.full(n, nd["y"], dtype=np.int64)
        xs, ys = [int(a) for a in x], [int(b) for b in y]
        f = {"add": lambda a, b: a + b, "sub": lambda a, b: a - b, "mul": lambda a, b: a * b}[nd["fn"]]
        out = dict(r)
        out[nd["out"]] = _wrap([f(a, b) for a, b in zip(xs, ys)])
        return out
    if op == "hash_join":
        r = _eval(plan, nd["input"], tables)
        s = _eval(plan, nd["build"], tables)
        index = {}
        for i, key in enumerate(s[nd["build_key"]]):
            if int(key) in index:
                raise DupKey(nd["build_key"])
            index[int(key)] = i
        pos = [index.get(int(key), -1) for key in r[nd["probe_key"]]]
        keep = np.array([p >= 0 for p in pos], dtype=bool)
        out = {c: v[keep] for c, v in r.items()}
        out[nd["payload"]] = s[nd["payload"]][[p for p in pos if p >= 0]].astype(np.int64)
        return out
    if op == "cross_join":
        r = _eval(plan, nd["input"], tables)
        s = _eval(plan, nd["right"], tables)
        n = len(next(iter(r.values())))
        m = len(next(iter(s.values())))
        out = {c: np.repeat(v, m) for c, v in r.items()}
        out.update({c: np.tile(v, n) for c, v in s.items()})
        return out
    raise ValueError(f"node {k}: {op} yields no relation below the root")


def run(tables: dict, plan: dict) -> dict:
    """The answer of the plan's root (a group_by or a project)."""
    nd = plan["nodes"][plan["root"]]
    r = _eval(plan, nd["input"], tables)
    n = len(next(iter(r.values()))) if r else 0
    if nd["op"] == "project":
        return {"kind": "project", "rows": n, "cols": [r[a].astype(np.int64) for a in nd["attrs"]]}
    assert nd["op"] == "group_by"
    keys = nd["keys"]
    groups = {}
    for i in range(n):
        groups.setdefault(tuple(int(r[g][i]) for g in keys), []).append(i)
    if not keys:
        groups.setdefault((), [])
    order = sorted(groups)
    out = {"kind": "aggregate", "rows": len(order),
           "keys": [np.array([k[j] for k in order], dtype=np.int64) for j in range(len(keys))],
           "count": np.array([len(groups[k]) for k in order], dtype=np.int64), "aggs": []}
    for fn, a, wide in nd["aggs"]:
        col = []
        for k in order:
            vals = [int(r[a][i]) for i in groups[k]] if a is not None else []
            if fn == "count":
                col.append(len(groups[k]))
            elif fn == "sum":
                t = sum(vals)
                col.append(t if wide else ((t + (1 << 63)) % M64) - (1 << 63))
            elif fn == "min":
                col.append(min(vals) if vals else (1 << 63) - 1)
            elif fn == "max":
                col.append(max(vals) if vals else -(1 << 63))
            elif fn == "avg":
                col.append(float(sum(vals)) / len(vals) if vals else float("nan"))
        if fn == "avg":
            out["aggs"].append(np.array(col, dtype=np.float64))
        elif fn == "sum" and wide:
            out["aggs"].append(np.array(col, dtype=object))
        else:
            out["aggs"].append(np.array(col, dtype=np.int64))
    return out
