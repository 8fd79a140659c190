"""GPU parity of relational plans: a plan compiled by the library's
produce/consume planner (hawk_query_from_plan) and run in several variants
gives the answer of the relational-plan oracle, which evaluates the plan node
by node without pipelines."""
import json
import os

import numpy as np
import pytest

from gpu_common import compare, say
from oracle import relalg
from paper_1709_00700_amd import hawk
from plans import random_case

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))

VARIANTS = [hawk.variant(proj_strategy=1, mem=1, pred=0, ht=0, hash=1, agg_strategy=0, thread_mult=8, wg_size=256),
            hawk.variant(proj_strategy=0, mem=0, pred=1, ht=1, hash=0, agg_strategy=1, thread_mult=1, wg_size=512),
            hawk.variant(proj_strategy=1, mem=0, pred=1, ht=1, hash=1, agg_strategy=0, thread_mult=1, wg_size=1024)]


@pytest.fixture
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hawk.Context(0)
    yield c
    c.close()


def spec_of(plan):
    """The root's description in the spec layout the result readers use."""
    root = plan["nodes"][plan["root"]]
    if root["op"] == "project":
        return {"main": {"project": root["attrs"]}}
    return {"main": {"group_by": root["keys"], "aggs": root["aggs"]}}


def check_plan(ctx, tables, plan, label):
    ref = relalg.run(tables, plan)
    ctx.register_numpy(tables)
    q = hawk.query_from_plan(ctx, plan)
    say(label, q.program().replace("\n", " | "))
    spec = spec_of(plan)
    for v in VARIANTS:
        r = hawk.execute(ctx, q, v)
        got = r.to_numpy(spec)
        r.free()
        compare(got, ref, spec, f"{label} {hawk.format_variant(v)}")
    return ref


def test_figure3_plan(ctx):
    with open(os.path.join(HERE, "golden", "plans", "figure3_two_joins.json")) as f:
        g = json.load(f)
    tables = {t: {c: np.array(v["values"], dtype=v["dtype"]) for c, v in cols.items()}
              for t, cols in g["tables"].items()}
    plan = g["plan"]
    for nd in plan["nodes"]:
        if "aggs" in nd:
            nd["aggs"] = [tuple(a) for a in nd["aggs"]]
    ref = check_plan(ctx, tables, plan, "figure 3")
    assert [int(x) for x in ref["aggs"][0]] == [900]


@pytest.mark.parametrize("seed", range(16))
def test_random_plans(ctx, seed):
    n = [0, 1, 65, 4097, 50_000, 200_000][seed % 6]
    tables, plan, _ = random_case(seed, n=n, prefix=f"g{seed}_")
    check_plan(ctx, tables, plan, f"plan {seed} n={n}")
