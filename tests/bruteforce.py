"""Row-at-a-time brute force for tiny tables: pins the oracle to the definitions.

Written independently of the oracle (different evaluation order, different
data structures): every fact row is pushed through the pipeline on its own, as
in the produce/consume model (Section 2.1); joins are nested loops over the
whole dimension (no map); groups are found by rescanning all surviving rows
for each distinct key; arithmetic uses Python integers reduced to 64-bit two's
complement; sums are exact Python integers and AVG an exact Fraction.
"""
from __future__ import annotations

from fractions import Fraction

M64 = 1 << 64


def to_i64(x: int) -> int:
    x %= M64
    return x - M64 if x >= 1 << 63 else x


def _passes(table, i, filters):
    for col, lo, hi in filters:
        v = int(table[col][i])
        if not (lo <= v <= hi):
            return False
    return True


def _build_rows(tables, b):
    """Dimension rows that pass the build pipeline's filters: list of (key, payload)."""
    t = tables[b["table"]]
    n = len(next(iter(t.values())))
    return [(int(t[b["key"]][i]), int(t[b["payload"]][i])) for i in range(n)
            if _passes(t, i, b.get("filters", []))]


def _row_attrs(tables, spec, i, dims, j=None):
    """Push fact row i (paired with row j of the CROSS_JOIN table, if any)
    through FILTER, CROSS_JOIN, FILTER, HASH_PROBE, ARITHMETIC; None if dropped."""
    m = spec["main"]
    t = tables[m["table"]]
    if not _passes(t, i, m.get("filters", [])):
        return None
    env = {c: int(t[c][i]) for c in t}
    if j is not None:
        u = tables[m["cross"]]
        env.update({c: int(u[c][j]) for c in u})
        for col, lo, hi in m.get("cross_filters", []):
            if not (lo <= env[col] <= hi):
                return None
    for fk, bi, pname in m.get("probes", []):
        matches = [pay for key, pay in dims[bi] if key == env[fk]]   # nested loop
        if not matches:
            return None
        assert len(matches) == 1, "dimension keys are unique"
        env[pname] = matches[0]
    for out, op, x, y in m.get("arith", []):
        xv = env[x] if isinstance(x, str) else int(x)
        yv = env[y] if isinstance(y, str) else int(y)
        env[out] = to_i64(xv + yv if op == "add" else xv - yv if op == "sub" else xv * yv)
    return env


def run(tables, spec):
    m = spec["main"]
    dims = [_build_rows(tables, b) for b in spec.get("builds", [])]
    for rows in dims:
        keys = [k for k, _ in rows]
        if len(set(keys)) != len(keys):
            return {"error": "dupkey"}
    t = tables[m["table"]]
    n = len(next(iter(t.values())))
    if m.get("cross"):
        # nested loops: the second table's rows vary fastest
        ni = len(next(iter(tables[m["cross"]].values())))
        cand = (_row_attrs(tables, spec, i, dims, j) for i in range(n) for j in range(ni))
    else:
        cand = (_row_attrs(tables, spec, i, dims) for i in range(n))
    envs = [e for e in cand if e is not None]
    if "project" in m:
        return {"kind": "project", "rows": len(envs),
                "cols": [[e[a] for e in envs] for a in m["project"]]}
    gb = m.get("group_by", [])
    distinct = sorted({tuple(e[g] for g in gb) for e in envs})
    if not gb:
        distinct = [()]
    out = {"kind": "aggregate", "rows": len(distinct), "keys": [[k[j] for k in distinct] for j in range(len(gb))],
           "count": [], "aggs": [[] for _ in m["aggs"]]}
    for key in distinct:
        members = [e for e in envs if tuple(e[g] for g in gb) == key]   # rescan for each group
        out["count"].append(len(members))
        for j, (fn, a, wide) in enumerate(m["aggs"]):
            vals = [e[a] for e in members] if a is not None else []
            if fn == "count":
                v = len(members)
            elif fn == "sum":
                v = sum(vals) if wide else to_i64(sum(vals))
            elif fn == "min":
                v = min(vals) if vals else (1 << 63) - 1
            elif fn == "max":
                v = max(vals) if vals else -(1 << 63)
            elif fn == "avg":
                v = Fraction(sum(vals), len(vals)) if vals else None
            out["aggs"][j].append(v)
    return out
