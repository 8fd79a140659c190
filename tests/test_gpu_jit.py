"""GPU parity of the grouped-aggregation kernels compiled at run time for each
plan structure: against the oracle, on the workloads' shapes (plain grouping,
spilling, joins, arithmetic with 128-bit sums, two group attributes), with
queries of one structure sharing their compiled kernel."""
import numpy as np
import pytest

from gpu_common import run_variants, sample, say
from paper_1709_00700_amd import datagen as dg
from paper_1709_00700_amd import hawk

pytestmark = pytest.mark.gpu


@pytest.fixture
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hawk.Context(0)
    c.set_jit(True)
    yield c
    c.close()


def lin_variants(ctx, tables, spec, k, seed):
    p = hawk.PlanningContext()
    p.register_shapes({t: {c: a[:1] for c, a in cols.items()} for t, cols in tables.items()})
    vs = [v for v in hawk.variant_space(hawk.build_query(p, spec)) if v.ht == 0]
    p.close()
    return sample(vs, k, seed)


@pytest.mark.parametrize("dist,nranks", [("uniform", 0), ("zipf", 60_000)])
def test_jit_group_aggregate(ctx, dist, nranks):
    kw = {"nranks": nranks} if nranks else {}
    tables, spec = dg.c2_aggregation(n=150_001, dist=dist, **kw)
    vs = lin_variants(ctx, tables, spec, 48, 11)
    say("jit c2", dist, len(vs))
    run_variants(ctx, tables, spec, vs, label=f"jit-{dist}")
    n, ms = ctx.jit_stats()
    assert n >= 1
    say("compiled", n, "kernels in", round(ms), "ms")


def test_jit_star_join(ctx):
    tables, spec = dg.c3_star_join(n=200_000, dims=(250, 2000, 300, 800), sel=(60, 50, 60, 40))
    run_variants(ctx, tables, spec, lin_variants(ctx, tables, spec, 24, 12), label="jit-c3")


def test_jit_wide_arithmetic(ctx):
    tables, spec = dg.c4_wide(n=100_003, price_hi=1 << 40)
    _, ref = run_variants(ctx, tables, spec, lin_variants(ctx, tables, spec, 24, 13), label="jit-c4")
    assert max(int(x) for x in ref["aggs"][4]) > (1 << 63)


def test_jit_two_keys_sentinel_and_spill(ctx):
    rng = np.random.default_rng(14)
    n = 120_000
    t = {"g1": rng.integers(-300, 300, size=n).astype(np.int32),
         "g2": rng.integers(-1, 40, size=n).astype(np.int32),
         "v": rng.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64),
         "f": rng.integers(0, 10, size=n).astype(np.int32)}
    spec = {"builds": [], "main": {"table": "t", "filters": [("f", 1, 8)], "probes": [],
                                   "arith": [("w", "sub", 0, "v")], "group_by": ["g1", "g2"],
                                   "aggs": [("sum", "v", True), ("sum", "w", True), ("min", "v", False),
                                            ("max", "w", False), ("avg", "v", True), ("count", None, False)],
                                   "groups_hint": 24_600}}
    run_variants(ctx, {"t": t}, spec, lin_variants(ctx, {"t": t}, spec, 32, 15), label="jit-wide-keys")


def test_jit_kernels_are_shared_by_one_structure(ctx):
    # two queries that differ only in data (tables, filter bounds) reuse one kernel
    v = hawk.variant(agg_strategy=0, ht=0, hash=1, mem=1, pred=0, thread_mult=8, wg_size=256)
    for i, (lo, hi) in enumerate([(0, 500_000), (100_000, 900_000)]):
        tables, spec = dg.c2_aggregation(n=50_000 + i, dist="uniform")
        tables = {f"t{i}": tables["t"]}
        spec["main"]["table"] = f"t{i}"
        spec["main"]["filters"] = [("v", lo, hi)]
        run_variants(ctx, tables, spec, [v], label=f"share{i}")
    assert ctx.jit_stats()[0] == 1


@pytest.mark.parametrize("n", [1, 4097, 1_000_000])
def test_jit_projection_every_multi_pass_variant(ctx, n):
    """The multi-pass filter and projection kernels compiled at run time for
    the plan: every multi-pass variant of C1, with the extra dimensions
    (unrolling, SIMD filter), against the oracle."""
    ctx.set_variant_dims(hawk.HAWK_DIM_UNROLL | hawk.HAWK_DIM_SIMD_FILTER)
    tables, spec = dg.c1_projection(n=n)
    tables = {f"jp{n}": tables["t"]}
    spec["main"]["table"] = f"jp{n}"
    p = hawk.PlanningContext()
    p.set_variant_dims(hawk.HAWK_DIM_UNROLL | hawk.HAWK_DIM_SIMD_FILTER)
    p.register_shapes(tables)
    vs = [v for v in hawk.variant_space(hawk.build_query(p, spec)) if v.proj_strategy == 1]
    p.close()
    k0 = ctx.jit_stats()[0]
    run_variants(ctx, tables, spec, vs, label=f"jit-proj n={n}")
    assert ctx.jit_stats()[0] > k0


def test_jit_projection_with_probes(ctx):
    tables, spec = dg.c3_star_join(n=30_000, dims=(50, 400, 60, 160), sel=(60, 50, 60, 40))
    spec["main"] = {"table": "f", "filters": [("rev", 0, 700_000)],
                    "probes": [("fk0", 0, "p0"), ("fk2", 2, "p2")],
                    "arith": [("x", "mul", "p0", "rev"), ("y", "sub", "x", "p2")],
                    "project": ["y", "fk0", "p2"]}
    spec["builds"] = spec["builds"][:3]
    vs = [hawk.variant(proj_strategy=1, mem=m, pred=pr, ht=h, hash=x, thread_mult=64)
          for m in (0, 1) for pr in (0, 1) for h in (0, 1, 2) for x in (0, 1)]
    ctx.set_variant_dims(hawk.HAWK_DIM_ROBIN_HOOD)
    run_variants(ctx, tables, spec, vs, label="jit-proj-join")


def test_jit_join_tables_in_lds_side_key_and_robin(ctx):
    # one small dimension: the run-time kernel copies its join table into
    # LDS (one workgroup per CU, and eight per CU) and probes it there; the
    # key -1 stays in the table's side word in device memory, and robin-hood
    # tables are probed from LDS as well. Fact keys 300..319 find no match.
    rng = np.random.default_rng(16)
    n = 90_001
    dk = np.arange(-1, 299, dtype=np.int32)
    rng.shuffle(dk)
    d = {"key": dk, "g": rng.integers(-3, 7, size=dk.size).astype(np.int32),
         "f": rng.integers(0, 10, size=dk.size).astype(np.int32)}
    d["f"][dk == -1] = 0  # key -1 passes the dimension's filter
    fact = {"fk": rng.integers(-1, 320, size=n).astype(np.int32),
            "v": rng.integers(-(1 << 40), 1 << 40, size=n, dtype=np.int64)}
    fact["fk"][::97] = -1
    spec = {"builds": [{"table": "d", "filters": [("f", 0, 6)], "key": "key", "payload": "g"}],
            "main": {"table": "f", "filters": [], "probes": [("fk", 0, "p0")], "arith": [],
                     "group_by": ["p0"], "aggs": [("sum", "v", False), ("count", None, False),
                                                  ("min", "v", False)],
                     "groups_hint": 10}}
    vs = [hawk.variant(agg_strategy=a, ht=ht, hash=h, mem=1, pred=p, thread_mult=tm, wg_size=wg)
          for ht in (hawk.HAWK_LINEAR_PROBING, hawk.HAWK_ROBIN_HOOD) for h in (0, 1) for p in (0, 1)
          for (a, tm, wg) in ((0, 1, 1024), (0, 8, 256), (1, 1, 512))]
    _, ref = run_variants(ctx, {"d": d, "f": fact}, spec, vs, label="jit-lds-join")
    assert -1 in set(int(k) for k in dk[d["f"] <= 6])


@pytest.mark.parametrize("shape", ["wide", "join"])
def test_jit_scalar_aggregate(ctx, shape):
    # AGGREGATE without grouping attributes through its run-time kernel: the
    # wide workload's arithmetic with 128-bit sums and a narrow AVG whose sum
    # passes 2^63, or a star join's probes; every sampled variant against the
    # oracle
    if shape == "wide":
        tables, spec = dg.c4_wide(n=100_003, price_hi=1 << 40)
        # the last aggregate becomes a narrow AVG of charge (about 2^53 per row)
        spec["main"]["aggs"] = list(spec["main"]["aggs"])[:-1] + [("avg", "charge", False)]
    else:
        tables, spec = dg.c3_star_join(n=150_000, dims=(250, 2000, 300, 800), sel=(60, 50, 60, 40))
        spec["main"]["aggs"] = [("sum", "rev", False), ("count", None, False), ("min", "rev", False),
                                ("max", "rev", False)]
    spec["main"]["group_by"] = []
    spec["main"].pop("groups_hint", None)
    before = ctx.jit_stats()[0]
    vs = lin_variants(ctx, tables, spec, 24, 17)
    say("jit scalar", shape, len(vs))
    run_variants(ctx, tables, spec, vs, label=f"jit-scalar-{shape}")
    assert ctx.jit_stats()[0] > before
