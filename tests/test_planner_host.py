"""Relational plans on the host (no GPU): the relational-plan oracle against
hand-worked values and against the pipeline oracle on the same queries
written as pipelines by hand; the library's produce/consume planner's
pipeline programs for the paper's two-join example, its pushdown of
selections, and its errors."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import relalg
from paper_1709_00700_amd import hawk
from plans import random_case

HERE = os.path.dirname(os.path.abspath(__file__))
FIG3 = os.path.join(HERE, "golden", "plans", "figure3_two_joins.json")


def load(path):
    with open(path) as f:
        g = json.load(f)
    tables = {t: {c: np.array(v["values"], dtype=v["dtype"]) for c, v in cols.items()}
              for t, cols in g["tables"].items()}
    plan = g["plan"]
    for nd in plan["nodes"]:
        if "aggs" in nd:
            nd["aggs"] = [tuple(a) for a in nd["aggs"]]
    return tables, plan, g


def as_py(r):
    out = {"rows": r["rows"]}
    if r["kind"] == "project":
        out["cols"] = [[int(x) for x in c] for c in r["cols"]]
    else:
        out["keys"] = [[int(x) for x in k] for k in r["keys"]]
        out["count"] = [int(x) for x in r["count"]]
        out["aggs"] = [[x if isinstance(x, float) else int(x) for x in a] for a in r["aggs"]]
    return out


def same(a, b):
    """Equal answers (AVG within 1e-12 relative)."""
    a, b = as_py(a), as_py(b)
    assert a["rows"] == b["rows"]
    if "cols" in a:
        assert a["cols"] == b["cols"]
        return
    assert a["keys"] == b["keys"] and a["count"] == b["count"]
    for x, y in zip(a["aggs"], b["aggs"]):
        for u, v in zip(x, y):
            if isinstance(u, float) or isinstance(v, float):
                assert (u != u and v != v) or abs(u - v) <= 1e-12 * abs(v)
            else:
                assert u == v


def test_relalg_figure3_hand_values():
    tables, plan, g = load(FIG3)
    r = as_py(relalg.run(tables, plan))
    e = g["expected"]
    assert r["rows"] == e["rows"] and r["keys"] == e["keys"] and r["count"] == e["count"]
    assert r["aggs"] == e["aggs"]


@pytest.mark.parametrize("seed", range(24))
def test_relalg_equals_pipeline_oracle(seed):
    """Two independent evaluations of one query: the plan node by node, and
    its pipelines (written by hand) column at a time."""
    tables, plan, spec = random_case(seed, n=int(np.random.default_rng(seed).integers(0, 400)))
    same(relalg.run(tables, plan), oracle.run(tables, spec))


@pytest.fixture
def plan_ctx():
    c = hawk.PlanningContext()
    yield c
    c.close()


def test_planner_figure3_program(plan_ctx):
    """The produce/consume partitioning of the two-join plan (Section 2.1)
    yields the pipeline programs of Table 2."""
    tables, plan, g = load(FIG3)
    plan_ctx.register_shapes(tables)
    q = hawk.query_from_plan(plan_ctx, plan)
    assert q.program().splitlines() == g["program"]
    assert q.kind == 2


def test_planner_pushes_selections_below_joins(plan_ctx):
    tables, plan, spec = random_case(3, n=50, prefix="q")
    plan_ctx.register_shapes(tables)
    # a selection on a scanned column above every join and the map
    nodes = list(plan["nodes"])
    root = nodes[plan["root"]]
    nodes.insert(len(nodes) - 1, {"op": "select", "input": root["input"], "attr": "v", "lo": -5, "hi": 5})
    nodes[-1] = dict(root, input=len(nodes) - 2)
    q = hawk.query_from_plan(plan_ctx, {"root": len(nodes) - 1, "nodes": nodes})
    probe = q.program().splitlines()[-1]
    later = [probe.find(op) for op in ("HASH_PROBE", "CROSS_JOIN", "ARITHMETIC") if op in probe]
    assert 0 < probe.find("FILTER(v in [-5, 5])") < min(later)


def test_planner_errors(plan_ctx):
    tables, plan, _ = load(FIG3)
    plan_ctx.register_shapes(tables)
    nodes = plan["nodes"]

    def expect(nodes, root, code):
        with pytest.raises(hawk.HawkError) as e:
            hawk.query_from_plan(plan_ctx, {"root": root, "nodes": nodes})
        assert e.value.code == code, e.value

    # a selection on a join's payload cannot move below the join
    bad = nodes[:8] + [{"op": "select", "input": 7, "attr": "x", "lo": 0, "hi": 9}, dict(nodes[8], input=8)]
    expect(bad, 9, hawk.HAWK_E_PLAN)
    # a build side with a join of its own
    bad = nodes[:8] + [{"op": "hash_join", "input": 5, "build": 6, "probe_key": "c", "build_key": "a",
                        "payload": "x"}, dict(nodes[8], input=8)]
    expect(bad, 9, hawk.HAWK_E_PLAN)
    # an aggregation below the root
    bad = nodes + [{"op": "project", "input": 8, "attrs": ["x"]}]
    expect(bad, 9, hawk.HAWK_E_PLAN)
    # a node that reaches itself, and a child index out of range
    bad = [dict(nd) for nd in nodes]
    bad[5] = dict(bad[5], input=6)
    expect(bad, 8, hawk.HAWK_E_PLAN)
    bad = [dict(nd) for nd in nodes]
    bad[6] = dict(bad[6], input=99)
    expect(bad, 8, hawk.HAWK_E_ARG)
    # the root is not a sink
    expect(nodes, 7, hawk.HAWK_E_PLAN)
