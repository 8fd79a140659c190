"""Random relational plans for the planner tests, each with the pipeline
decomposition written out by hand beside it.

`random_case(seed, n)` draws a fact table of n rows and up to three
dimension tables with unique keys, and builds both
  * a relational plan (the format of oracle.relalg): scans, selections above
    and below the joins, hash joins whose build sides are filtered scans, a
    map, optionally a cross join with a small table, and a group-by or
    projection at the root; and
  * the same query as build pipelines plus one probe pipeline (the spec
    format of the pipeline oracle), written directly from the operators.
The plan's answer (oracle.relalg) and the spec's (oracle.run) must agree;
the library's planner then has to reproduce that answer from the plan alone.
"""
from __future__ import annotations

import numpy as np

from paper_1709_00700_amd import datagen as dg

I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1


def random_case(seed: int, n: int, prefix: str = "p"):
    rng = np.random.default_rng(seed)
    s = dg.MASTER_SEED + 9000 + seed
    t = {}
    fact = f"{prefix}f"
    t[fact] = {"a": dg.uniform(s, 1, n, -50, 50, np.int32),
               "v": dg.uniform(s, 2, n, -(1 << 40), 1 << 40, np.int64),
               "w": dg.uniform(s, 3, n, -4, 5, np.int8)}
    nodes = [{"op": "scan", "table": fact}]
    cur = 0
    spec_main = {"table": fact, "filters": [], "probes": [], "arith": []}
    builds = []
    # a selection below the joins
    if rng.random() < 0.7:
        nodes.append({"op": "select", "input": cur, "attr": "a", "lo": -40, "hi": int(rng.integers(0, 50))})
        cur = len(nodes) - 1
        spec_main["filters"].append(("a", -40, nodes[-1]["hi"]))
    njoin = int(rng.integers(0, 4))
    late = []  # selections placed above the joins (on fact columns)
    for j in range(njoin):
        nd = int(rng.integers(1, 60))
        dim = f"{prefix}d{j}"
        t[dim] = {f"k{j}": dg.sparse_keys(s, 10 + j, nd),
                  f"f{j}": dg.uniform(s, 20 + j, nd, 0, 10, np.int32),
                  f"g{j}": dg.uniform(s, 30 + j, nd, -3, 4, np.int32)}
        t[fact][f"fk{j}"] = dg.foreign_keys(s, 40 + j, 10 + j, n, nd)
        scan = len(nodes)
        nodes.append({"op": "scan", "table": dim})
        fhi = int(rng.integers(2, 10))
        nodes.append({"op": "select", "input": scan, "attr": f"f{j}", "lo": 0, "hi": fhi})
        nodes.append({"op": "hash_join", "input": cur, "build": scan + 1, "probe_key": f"fk{j}",
                      "build_key": f"k{j}", "payload": f"g{j}"})
        cur = len(nodes) - 1
        builds.append({"table": dim, "filters": [(f"f{j}", 0, fhi)], "key": f"k{j}", "payload": f"g{j}"})
        spec_main["probes"].append((f"fk{j}", j, f"g{j}"))
        if rng.random() < 0.4:
            late.append(("w", -3, int(rng.integers(0, 5))))
    for col, lo, hi in late:
        nodes.append({"op": "select", "input": cur, "attr": col, "lo": lo, "hi": hi})
        cur = len(nodes) - 1
        spec_main["filters"].append((col, lo, hi))
    cross = rng.random() < 0.35
    if cross:
        m = int(rng.integers(1, 12))
        u = f"{prefix}u"
        t[u] = {"b": dg.uniform(s, 50, m, -5, 5, np.int32), "e": dg.uniform(s, 51, m, -9, 10, np.int64)}
        scan = len(nodes)
        nodes.append({"op": "scan", "table": u})
        nodes.append({"op": "select", "input": scan, "attr": "b", "lo": -4, "hi": 3})
        nodes.append({"op": "cross_join", "input": cur, "right": scan + 1})
        cur = len(nodes) - 1
        spec_main["cross"] = u
        spec_main["cross_filters"] = [("b", -4, 3)]
    nodes.append({"op": "map", "input": cur, "out": "vw", "fn": "mul", "x": "v", "y": "w"})
    cur = len(nodes) - 1
    spec_main["arith"].append(("vw", "mul", "v", "w"))
    gattr = (["g0"] if njoin else ["w"]) + (["b"] if cross else [])
    if rng.random() < 0.5:
        attrs = ["vw", "a"] + ([f"g{njoin - 1}"] if njoin else []) + (["e"] if cross else [])
        nodes.append({"op": "project", "input": cur, "attrs": attrs})
        spec_main["project"] = attrs
    else:
        aggs = [("count", None, False), ("sum", "vw", True), ("min", "v", False), ("max", "a", False),
                ("avg", "vw", False)]
        nodes.append({"op": "group_by", "input": cur, "keys": gattr, "aggs": aggs, "groups_hint": 256})
        spec_main.update(group_by=gattr, aggs=aggs, groups_hint=256)
    plan = {"root": len(nodes) - 1, "nodes": nodes}
    return t, plan, {"builds": builds, "main": spec_main}
