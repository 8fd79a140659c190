"""GPU parity of the extra variant dimensions (hawk_ctx_set_variant_dims):
robin-hood join tables (the extension of Section 7.5.1), the SIMD filter
(Section 7.5.2) and loop unrolling (Section 6.1), each against the oracle
element by element, on ragged sizes and the edge cases of each."""
import numpy as np
import pytest

import oracle
from gpu_common import run_variants, sample, say
from paper_1709_00700_amd import datagen as dg
from paper_1709_00700_amd import hawk

pytestmark = pytest.mark.gpu

ALL = hawk.HAWK_DIM_ROBIN_HOOD | hawk.HAWK_DIM_UNROLL | hawk.HAWK_DIM_SIMD_FILTER


@pytest.fixture
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hawk.Context(0)
    c.set_variant_dims(ALL)
    yield c
    c.close()


def space(tables, spec):
    plan = hawk.PlanningContext()
    plan.set_variant_dims(ALL)
    plan.register_shapes(tables)
    vs = hawk.variant_space(hawk.build_query(plan, spec))
    plan.close()
    return vs


def renamed(tables, spec, p):
    t = {p + k: v for k, v in tables.items()}
    s = {"builds": [dict(b, table=p + b["table"]) for b in spec["builds"]], "main": dict(spec["main"])}
    s["main"]["table"] = p + s["main"]["table"]
    return t, s


# ------------------------------------------------------------------ robin hood
def test_robin_hood_star_join(ctx):
    tables, spec = renamed(*dg.c3_star_join(n=200_000, dims=(250, 20_000, 300, 800), sel=(60, 50, 60, 40)), "rh_")
    vs = [v for v in space(tables, spec) if v.ht == hawk.HAWK_ROBIN_HOOD]
    assert len(vs) == 896 // 4 * 2
    say("robin hood, star join", len(vs))
    run_variants(ctx, tables, spec, sample(vs, 64, seed=4), label="robin c3")


def test_robin_hood_projection_and_sentinel_keys(ctx):
    d = {"key": np.array([-1, 5, -(1 << 31), (1 << 31) - 1, 7, 0], np.int32),
         "g": np.array([10, 20, 30, 40, 50, -1], np.int32)}
    rng = np.random.default_rng(5)
    f = {"fk": rng.choice(np.array([-1, 5, -(1 << 31), (1 << 31) - 1, 7, 0, 3, -2], np.int32), size=5000),
         "v": rng.integers(0, 100, size=5000).astype(np.int64)}
    spec = {"builds": [{"table": "rk_d", "filters": [], "key": "key", "payload": "g"}],
            "main": {"table": "rk_f", "filters": [], "probes": [("fk", 0, "p")], "arith": [], "project": ["p", "v"]}}
    tables = {"rk_d": d, "rk_f": f}
    vs = [v for v in space(tables, spec) if v.ht == hawk.HAWK_ROBIN_HOOD]
    run_variants(ctx, tables, spec, vs, label="robin keys")


def test_robin_hood_dense_table_and_duplicates(ctx):
    # 40k distinct keys into a table of 2^17 slots; then a key inserted twice
    tables, spec = renamed(*dg.c3_star_join(n=100_000, dims=(40_000, 50, 60, 70), sel=(100, 100, 100, 100)), "rd_")
    run_variants(ctx, tables, spec, [hawk.variant(ht=2, hash=h, agg_strategy=s, thread_mult=8, wg_size=256)
                                     for h in (0, 1) for s in (0, 1)], label="robin dense")
    d = {"key": np.array([3, 9, 3, 4], np.int32), "g": np.array([1, 2, 3, 4], np.int32)}
    f = {"fk": np.array([3, 4, 9], np.int32)}
    spec = {"builds": [{"table": "rdd", "filters": [], "key": "key", "payload": "g"}],
            "main": {"table": "rdf", "filters": [], "probes": [("fk", 0, "p")], "arith": [], "project": ["p"]}}
    ctx.register_numpy({"rdd": d, "rdf": f})
    q = hawk.build_query(ctx, spec)
    with pytest.raises(hawk.HawkError) as e:
        hawk.execute(ctx, q, hawk.variant(ht=2))
    assert e.value.code == hawk.HAWK_E_DUPKEY


def test_robin_hood_in_a_batch(ctx):
    tables, spec = renamed(*dg.c3_star_join(n=50_000, dims=(250, 2000, 300, 800), sel=(60, 50, 60, 40)), "rb_")
    ref = oracle.run(tables, spec)
    ctx.register_numpy(tables)
    q = hawk.build_query(ctx, spec)
    b = hawk.Batch(ctx, [q], variants=[hawk.variant(ht=2, hash=1, thread_mult=8, wg_size=256)])
    b.run()
    b.run()
    r = b.result(0)
    got = r.to_numpy(spec)
    r.free()
    b.free()
    from gpu_common import compare
    compare(got, ref, spec, "robin batch")


# ------------------------------------------------------------------ SIMD filter and unrolling
@pytest.mark.parametrize("n", [1, 63, 255, 256, 257, 4097, 1_000_000])
def test_simd_filter_and_unrolling_c1(ctx, n):
    tables, spec = renamed(*dg.c1_projection(n=n), f"sf{n}_")
    vs = [v for v in space(tables, spec) if v.filter_mode or v.unroll]
    assert len(vs) == 14 * 3
    run_variants(ctx, tables, spec, vs, label=f"simd/unroll n={n}")


def test_simd_filter_int8_int64_columns(ctx):
    n = 70_001
    t = {"a8": dg.uniform(dg.MASTER_SEED, 0x8001, n, -128, 128, np.int8),
         "b64": dg.uniform(dg.MASTER_SEED, 0x8002, n, -(1 << 40), 1 << 40, np.int64),
         "c": dg.uniform(dg.MASTER_SEED, 0x8003, n, -1000, 1000, np.int32)}
    spec = {"builds": [], "main": {"table": "s8", "filters": [("a8", -100, 30), ("b64", -(1 << 39), 1 << 38),
                                                              ("c", -900, 800)],
                                   "probes": [], "arith": [("x", "add", "b64", "c")], "project": ["x", "a8"]}}
    vs = [v for v in space({"s8": t}, spec) if v.filter_mode]
    run_variants(ctx, {"s8": t}, spec, vs, label="simd i8/i64")


def test_simd_filter_needs_aligned_columns(ctx):
    import torch
    n = 10_000
    a = torch.arange(n + 1, dtype=torch.int32, device="cuda")
    ctx.register("mis", {"a": a[1:], "b": a[1:]})   # 4 bytes past a 16-byte boundary
    spec = {"builds": [], "main": {"table": "mis", "filters": [("a", 0, 500)], "probes": [], "arith": [],
                                   "project": ["b"]}}
    q = hawk.build_query(ctx, spec)
    with pytest.raises(hawk.HawkError) as e:
        hawk.execute(ctx, q, hawk.variant(proj_strategy=1, mem=1, thread_mult=8, filter_mode=1))
    assert e.value.code == hawk.HAWK_E_INFEASIBLE
    r = hawk.execute(ctx, q, hawk.variant(proj_strategy=1, mem=1, thread_mult=8, unroll=2))
    assert r.info()[0] == 500
    r.free()
