"""GPU parity: every variant of the HIP path against the CPU oracle, through
the C ABI, on seeded inputs that span several tiles and a ragged tail, plus
the degenerate cases of the method."""
import numpy as np
import pytest

import oracle
from gpu_common import compare, run_variants, sample, say
from paper_1709_00700_amd import datagen as dg
from paper_1709_00700_amd import hawk

pytestmark = pytest.mark.gpu


@pytest.fixture
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hawk.Context(0)
    yield c
    c.close()


def all_variants(ctx, tables, spec):
    p = hawk.PlanningContext()
    p.register_shapes({t: {c: a[:1] for c, a in cols.items()} for t, cols in tables.items()})
    vs = hawk.variant_space(hawk.build_query(p, spec))
    p.close()
    return vs


# ------------------------------------------------------------------ projection
@pytest.mark.parametrize("n", [1_000_000, 100_003])
def test_c1_all_32_variants(ctx, n):
    tables, spec = dg.c1_projection(n=n)
    vs = all_variants(ctx, tables, spec)
    assert len(vs) == 32
    say("c1 n", n)
    run_variants(ctx, tables, spec, vs, label="c1")


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 4097])
def test_c1_small_and_ragged(ctx, n):
    tables, spec = dg.c1_projection(n=n)
    say("c1 ragged n", n)
    run_variants(ctx, tables, spec, all_variants(ctx, tables, spec), label=f"c1 n={n}")


@pytest.mark.parametrize("which", ["all", "none"])
def test_c1_all_or_none_selected(ctx, which):
    tables, spec = dg.c1_projection(n=20_000)
    spec["main"]["filters"] = [("a", 0, 999)] if which == "all" else [("a", 5000, 6000)]
    say("c1", which)
    run_variants(ctx, tables, spec, all_variants(ctx, tables, spec), label=f"c1 {which}")


def test_projection_with_join_probe(ctx):
    tables, spec = dg.c3_star_join(n=30_000, dims=(50, 400, 60, 160), sel=(60, 50, 60, 40))
    spec["main"] = {"table": "f", "filters": [("rev", 0, 700_000)],
                    "probes": [("fk0", 0, "p0"), ("fk2", 2, "p2")],
                    "arith": [("x", "mul", "p0", "rev"), ("y", "sub", "x", "p2")],
                    "project": ["y", "fk0", "p2"]}
    spec["builds"] = [spec["builds"][0], spec["builds"][1], spec["builds"][2]]
    vs = all_variants(ctx, tables, spec)
    assert len(vs) == 128
    say("projection with probes")
    run_variants(ctx, tables, spec, vs, label="proj-join")


# ------------------------------------------------------------------ grouped aggregation
def test_c2_uniform_all_896_variants(ctx):
    tables, spec = dg.c2_aggregation(n=50_003, dist="uniform")
    vs = all_variants(ctx, tables, spec)
    assert len(vs) == 896
    say("c2 uniform, 896 variants")
    run_variants(ctx, tables, spec, vs, label="c2u")


def test_c2_zipf_sampled_variants(ctx):
    tables, spec = dg.c2_aggregation(n=300_007, dist="zipf", nranks=200_000)
    vs = sample(all_variants(ctx, tables, spec), 96, seed=1)
    say("c2 zipf, 96 variants")
    run_variants(ctx, tables, spec, vs, label="c2z")


def local_linear(vs):
    return [v for v in vs if v.agg_strategy == 0 and v.ht == 0]


def test_overflow_partitioning_all_local_linear_variants(ctx):
    # 60k zipf ranks: far more groups than an LDS table holds, so every local
    # linear-probing variant spills its LDS misses and aggregates them per region
    tables, spec = dg.c2_aggregation(n=150_001, dist="zipf", nranks=60_000)
    vs = local_linear(all_variants(ctx, tables, spec))
    assert len(vs) == 392
    say("overflow partitioning, 392 variants")
    run_variants(ctx, tables, spec, vs, label="spill")


def test_overflow_partitioning_wide_sums_two_keys(ctx):
    rng = np.random.default_rng(12)
    n = 120_000
    t = {"g1": rng.integers(-300, 300, size=n).astype(np.int32),
         "g2": rng.integers(-1, 40, size=n).astype(np.int32),
         "v": rng.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64),
         "f": rng.integers(0, 10, size=n).astype(np.int32)}
    spec = {"builds": [], "main": {"table": "t", "filters": [("f", 1, 8)], "probes": [],
                                   "arith": [("w", "sub", 0, "v")],
                                   "group_by": ["g1", "g2"],
                                   "aggs": [("sum", "v", True), ("sum", "w", True), ("min", "v", False),
                                            ("max", "w", False), ("avg", "v", True), ("count", None, False)],
                                   "groups_hint": 24_600}}
    vs = sample(local_linear(all_variants(ctx, {"t": t}, spec)), 64, seed=7)
    say("overflow partitioning: two keys, 128-bit sums, AVG")
    _, ref = run_variants(ctx, {"t": t}, spec, vs, label="spill-wide")
    assert ref["rows"] > 20_000


@pytest.mark.parametrize("aggs", [[("count", None, False), ("sum", "v", False), ("min", "v", False),
                                   ("max", "v", False)],
                                  [("count", None, False)]])
def test_overflow_partitioning_one_hot_region(ctx, aggs):
    # The first half of the rows (in scan order) cycles over 300k keys, so a
    # workgroup's LDS table is full before the second half, which holds one
    # key only, begins. On a coalesced grid every workgroup then spills that
    # key's rows, so one table region receives half of all rows and its owner
    # aggregates 1.2M entries on one slot. COUNT alone spills keys without values.
    rng = np.random.default_rng(31)
    n = 2_400_000
    key = np.empty(n, np.int32)
    key[:n // 2] = (np.arange(n // 2) % 300_000) + 1
    key[n // 2:] = -5
    t = {"g": key, "v": rng.integers(-(1 << 40), 1 << 40, size=n, dtype=np.int64)}
    spec = {"builds": [], "main": {"table": "t", "filters": [], "probes": [], "arith": [],
                                   "group_by": ["g"], "aggs": aggs, "groups_hint": 300_001}}
    vs = [v for v in local_linear(all_variants(ctx, {"t": t}, spec))
          if v.mem == 1 and v.thread_mult <= 2 and v.wg_size >= 256]
    vs = sample(vs, 16, seed=9)
    say("overflow partitioning, one hot region", len(aggs), "aggregates")
    _, ref = run_variants(ctx, {"t": t}, spec, vs, label="spill-one-region")
    assert ref["rows"] == 300_001


def test_c3_star_join_sampled_variants(ctx):
    tables, spec = dg.c3_star_join(n=200_000, dims=(250, 2000, 300, 800), sel=(60, 50, 60, 40))
    vs = sample(all_variants(ctx, tables, spec), 128, seed=2)
    say("c3, 128 variants")
    run_variants(ctx, tables, spec, vs, label="c3")


def test_c4_wide_sampled_variants(ctx):
    tables, spec = dg.c4_wide(n=100_003, price_hi=1 << 40)
    vs = sample(all_variants(ctx, tables, spec), 96, seed=3)
    say("c4, 96 variants")
    _, ref = run_variants(ctx, tables, spec, vs, label="c4")
    assert max(int(x) for x in ref["aggs"][4]) > (1 << 63)   # the wide sum really needs 128 bits


def test_scalar_aggregate_all_variants(ctx):
    tables, spec = dg.c4_wide(n=70_001)
    spec["main"]["group_by"] = []
    spec["main"]["filters"] = [("qty", 10, 40)]
    vs = all_variants(ctx, tables, spec)
    assert len(vs) == 224
    say("aggregate without groups, 224 variants")
    run_variants(ctx, tables, spec, vs, label="agg")


def test_scalar_aggregate_empty_input(ctx):
    tables, spec = dg.c4_wide(n=1000)
    spec["main"]["group_by"] = []
    spec["main"]["filters"] = [("qty", 100, 200)]     # nothing qualifies
    run_variants(ctx, tables, spec, sample(all_variants(ctx, tables, spec), 16), label="agg-empty")


def test_negative_and_overflowing_sums(ctx):
    rng = np.random.default_rng(11)
    n = 40_000
    t = {"g1": rng.integers(-2, 2, size=n).astype(np.int8),
         "g2": rng.integers(-3, 1, size=n).astype(np.int32),
         "v": rng.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64) * 2 + 1,
         "f": rng.integers(0, 10, size=n).astype(np.int32)}
    spec = {"builds": [], "main": {"table": "t", "filters": [("f", 2, 8)], "probes": [],
                                   "arith": [("w", "sub", 0, "v")],
                                   "group_by": ["g1", "g2"],
                                   "aggs": [("sum", "v", True), ("sum", "w", True), ("sum", "v", False),
                                            ("min", "v", False), ("max", "w", False), ("avg", "v", True),
                                            ("count", None, False)],
                                   "groups_hint": 16}}
    vs = sample(all_variants(ctx, {"t": t}, spec), 96, seed=4)
    # the group (-1, -1) packs to the all-ones key and takes the side slot
    say("sentinel groups + 128-bit sums")
    _, ref = run_variants(ctx, {"t": t}, spec, vs, label="wide")
    assert any(k0 == -1 and k1 == -1 for k0, k1 in zip(ref["keys"][0], ref["keys"][1]))


def test_join_key_minus_one_and_sparse_keys(ctx):
    d = {"key": np.array([-1, 5, -(1 << 31), (1 << 31) - 1, 7, 0], np.int32),
         "g": np.array([10, 20, 30, 40, 50, -1], np.int32)}
    rng = np.random.default_rng(5)
    f = {"fk": rng.choice(np.array([-1, 5, -(1 << 31), (1 << 31) - 1, 7, 0, 3, -2], np.int32), size=5000),
         "v": rng.integers(0, 100, size=5000).astype(np.int64)}
    spec = {"builds": [{"table": "d", "filters": [], "key": "key", "payload": "g"}],
            "main": {"table": "f", "filters": [], "probes": [("fk", 0, "p")], "arith": [],
                     "group_by": ["p"], "aggs": [("sum", "v", False), ("count", None, False)], "groups_hint": 8}}
    vs = sample(all_variants(ctx, {"d": d, "f": f}, spec), 64, seed=6)
    run_variants(ctx, {"d": d, "f": f}, spec, vs, label="keys")


@pytest.mark.parametrize("ht", [0, 1])
def test_duplicate_build_key_is_reported(ctx, ht):
    d = {"key": np.array([3, 9, 3, 4], np.int32), "g": np.array([1, 2, 3, 4], np.int32)}
    f = {"fk": np.array([3, 4, 9], np.int32)}
    spec = {"builds": [{"table": "d", "filters": [], "key": "key", "payload": "g"}],
            "main": {"table": "f", "filters": [], "probes": [("fk", 0, "p")], "arith": [], "project": ["p"]}}
    ctx.register_numpy({"d": d, "f": f})
    q = hawk.build_query(ctx, spec)
    with pytest.raises(hawk.HawkError) as e:
        hawk.execute(ctx, q, hawk.variant(ht=ht))
    assert e.value.code == hawk.HAWK_E_DUPKEY


def test_undersized_group_hint_retries(ctx):
    tables, spec = dg.c2_aggregation(n=60_000, dist="uniform", groups=3000)
    spec["main"]["groups_hint"] = 40          # table for 80 slots, 3000 groups arrive
    vs = [hawk.variant(agg_strategy=s, ht=h, hash=x, mem=1, thread_mult=8, wg_size=256)
          for s in (0, 1) for h in (0, 1) for x in (0, 1)]
    run_variants(ctx, tables, spec, vs, label="hint")


def test_async_execution_matches(ctx):
    tables, spec = dg.c2_aggregation(n=100_000, dist="zipf", nranks=5000)
    ref = oracle.run(tables, spec)
    ctx.register_numpy(tables)
    q = hawk.build_query(ctx, spec)
    rs = [hawk.execute(ctx, q, hawk.variant(agg_strategy=i % 2, ht=i // 2 % 2), sync=False) for i in range(4)]
    for r in rs:
        compare(r.to_numpy(spec), ref, spec, "async")
        r.free()


# ------------------------------------------------------------------ AVG of sums beyond 64 bits
def _avg_overflow_table(n, ngroups, seed):
    # every value lies in [2^62 - 2^40, 2^62) or its negation: any two rows of
    # one sign already sum past 2^63, so a 64-bit accumulator would wrap
    rng = np.random.default_rng(seed)
    mag = rng.integers((1 << 62) - (1 << 40), 1 << 62, size=n, dtype=np.int64)
    sign = np.where(rng.integers(0, 8, size=n) == 0, -1, 1).astype(np.int64)
    t = {"g": rng.integers(0, ngroups, size=n).astype(np.int32) * 7919 - 3,
         "v": mag * sign,
         "q": rng.integers(-50, 50, size=n).astype(np.int32)}
    aggs = [("avg", "v", False), ("count", None, False), ("sum", "v", False), ("avg", "q", False)]
    return t, aggs


@pytest.mark.parametrize("ngroups", [16, 40_000, 0])
def test_narrow_avg_of_overflowing_sum(ctx, ngroups):
    """AVG(v) with wide=0 divides the exact sum (the oracle's reading), on the
    local/global, linear/cuckoo, spilling and non-grouped paths."""
    t, aggs = _avg_overflow_table(90_001, max(ngroups, 1), 21 + ngroups % 97)
    spec = {"builds": [], "main": {"table": "t", "filters": [("q", -45, 45)], "probes": [], "arith": [],
                                   "group_by": ["g"] if ngroups else [], "aggs": aggs,
                                   "groups_hint": max(ngroups, 1)}}
    ref = oracle.run({"t": t}, spec)
    # the exact per-group sums really leave the int64 range
    assert any(abs(a * c) > (1 << 63) for a, c in zip(ref["aggs"][0], ref["count"]) if c)
    vs = all_variants(ctx, {"t": t}, spec)
    picked = sample(vs, 48, seed=ngroups + 1)
    if ngroups >= 10_000:
        picked += sample(local_linear(vs), 24, seed=5)   # spilling variants
    say("narrow AVG of overflowing sums, groups", ngroups, "variants", len(picked))
    run_variants(ctx, {"t": t}, spec, picked, ref=ref, label=f"avg{ngroups}")


def test_narrow_avg_run_time_kernel_and_batch(ctx):
    t, aggs = _avg_overflow_table(120_003, 30_000, 77)
    spec = {"builds": [], "main": {"table": "t", "filters": [], "probes": [], "arith": [],
                                   "group_by": ["g"], "aggs": aggs, "groups_hint": 30_000}}
    ref = oracle.run({"t": t}, spec)
    ctx.set_jit(True)
    vs = [hawk.variant(agg_strategy=s, ht=0, hash=h, mem=1, pred=p, thread_mult=tm, wg_size=wg)
          for s, h, p, tm, wg in [(0, 1, 0, 1, 1024), (0, 0, 1, 8, 256), (1, 1, 0, 1, 512), (0, 1, 1, 64, 128)]]
    say("narrow AVG: run-time compiled kernels")
    q, _ = run_variants(ctx, {"t": t}, spec, vs, ref=ref, label="avg-jit")
    assert ctx.jit_stats()[0] >= 1
    say("narrow AVG: batch")
    for sep in (0, 1):
        b = hawk.Batch(ctx, [q], separate=sep)
        b.run()
        r = b.result(0)
        compare(r.to_numpy(spec), ref, spec, f"avg-batch separate={sep}")
        r.free()
        b.free()


@pytest.mark.parametrize("sink", ["project", "group"])
def test_cross_join_variants(ctx, sink):
    """CROSS_JOIN (Table 1): 20k x 64 pairs (a filter on each side, a band
    filter on the pair, a probe keyed by the second table, arithmetic over
    both), projection in (row, second-table row) order or grouping, in every
    projection variant or a sample of the aggregation variants."""
    tables, spec = dg.cross_join(n=20_000, m=64, sink=sink)
    tables = {f"x{sink}_{t}": c for t, c in tables.items()}
    spec["main"]["table"] = f"x{sink}_t"
    spec["main"]["cross"] = f"x{sink}_u"
    spec["builds"][0]["table"] = f"x{sink}_d"
    plan = hawk.PlanningContext()
    plan.register_shapes(tables)
    vs = hawk.variant_space(hawk.build_query(plan, spec))
    plan.close()
    say("cross join", sink, "variants", len(vs))
    run_variants(ctx, tables, spec, vs if sink == "project" else sample(vs, 48, seed=5), label=f"cross {sink}")


def test_cross_join_ragged_and_empty(ctx):
    for i, (n, m) in enumerate([(1, 1), (63, 1), (65, 3), (0, 5), (7, 0), (4097, 17)]):
        tables, spec = dg.cross_join(n=n, m=m, nd=5, sink="project" if i % 2 else "group")
        tables = {f"xr{i}_{t}": c for t, c in tables.items()}
        spec["main"]["table"], spec["main"]["cross"] = f"xr{i}_t", f"xr{i}_u"
        spec["builds"][0]["table"] = f"xr{i}_d"
        run_variants(ctx, tables, spec, [hawk.variant(proj_strategy=1, thread_mult=8),
                                          hawk.variant(agg_strategy=1, ht=1, wg_size=64)], label=f"cross {n}x{m}")
