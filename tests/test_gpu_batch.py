"""GPU parity of batched execution: a mixed workload of projection,
aggregation and star-join pipelines replayed as one captured graph of
persistent kernels, every query's result against the oracle, over several
replays, schedules and the autotuner's re-capture."""
import numpy as np
import pytest

import oracle
from gpu_common import compare, say
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


def c5_setup(ctx, nq, pool_rows, min_rows, max_rows, seed=dg.MASTER_SEED + 5):
    """Registers the pools once on the device and every query's window as a
    table of views into them; returns (queries, handles, oracle answers)."""
    import torch
    pools = dg.c5_pools(pool_rows, seed)
    qs = dg.c5_queries(nq, pool_rows, seed, min_rows=min_rows, max_rows=max_rows)
    dev = {p: {c: torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for c, a in cols.items()}
           for p, cols in pools.items()}
    for j in range(4):
        ctx.register(f"d{j}", dev[f"d{j}"])
    handles, refs = [], []
    for q in qs:
        o, n = q["offset"], q["rows"]
        ctx.register(q["window"], {c: t[o:o + n] for c, t in dev[q["pool"]].items()})
        handles.append(hawk.build_query(ctx, q["spec"]))
        refs.append(oracle.run(dg.c5_window_tables(pools, q), q["spec"]))
    ctx._keep.append(dev)
    return qs, handles, refs


def check_batch(b, qs, refs, label):
    for i, (q, ref) in enumerate(zip(qs, refs)):
        r = b.result(i)
        got = r.to_numpy(q["spec"])
        r.free()
        compare(got, ref, q["spec"], f"{label} query {i} kind {q['kind']} rows {q['rows']}")


def test_batch_mixed_workload_two_replays(ctx):
    say("batch: 24 mixed queries, up to 400k rows each")
    qs, hs, refs = c5_setup(ctx, 24, 400_000, 1000, 400_000)
    assert {q["kind"] for q in qs} == {1, 2, 3}
    b = hawk.Batch(ctx, hs)
    for rep in range(2):
        b.run()
        check_batch(b, qs, refs, f"replay {rep}")
    b.free()


@pytest.mark.parametrize("tile,wgs,order", [(14, 1, 0), (18, 8, 1), (15, 3, 0)])
def test_batch_schedules(ctx, tile, wgs, order):
    say("batch schedule", tile, wgs, order)
    qs, hs, refs = c5_setup(ctx, 12, 300_000, 1000, 300_000, seed=dg.MASTER_SEED + 55)
    b = hawk.Batch(ctx, hs, tile_rows_log2=tile, wgs_per_cu=wgs, order=order)
    assert b.opts() == {"tile_rows_log2": tile, "wgs_per_cu": wgs, "order": order, "separate": 1}
    b.run()
    check_batch(b, qs, refs, f"tile {tile} wgs {wgs} order {order}")
    b.free()


def test_batch_without_separate_launches(ctx):
    say("batch: every pipeline in the persistent kernels")
    qs, hs, refs = c5_setup(ctx, 12, 2_000_000, 1_000_000, 2_000_000, seed=dg.MASTER_SEED + 59)
    b = hawk.Batch(ctx, hs, separate=0)
    b.run()
    check_batch(b, qs, refs, "no separate launches")
    b.free()


def test_batch_separate_launches_large_groups(ctx):
    # pipelines of 1M-2M rows: the high-cardinality aggregations get their own launches
    say("batch: separate launches")
    qs, hs, refs = c5_setup(ctx, 12, 2_000_000, 1_000_000, 2_000_000, seed=dg.MASTER_SEED + 59)
    assert any(q["kind"] == 2 and q["groups"] >= 4096 for q in qs)
    b = hawk.Batch(ctx, hs, separate=1)
    for rep in range(2):
        b.run()
        check_batch(b, qs, refs, f"separate, replay {rep}")
    b.free()


def test_batch_tiny_ragged_queries(ctx):
    # windows of 1..5000 rows: single partial tiles, empty selections, one-row groups
    say("batch: 32 tiny queries")
    qs, hs, refs = c5_setup(ctx, 32, 50_000, 1, 5000, seed=dg.MASTER_SEED + 56)
    b = hawk.Batch(ctx, hs, tile_rows_log2=14, wgs_per_cu=2)
    b.run()
    b.run()
    check_batch(b, qs, refs, "tiny")
    b.free()


def test_batch_autotune_recaptures(ctx):
    say("batch autotune")
    qs, hs, refs = c5_setup(ctx, 8, 200_000, 1000, 200_000, seed=dg.MASTER_SEED + 57)
    b = hawk.Batch(ctx, hs)
    best, ms = b.autotune(reps=1)
    assert b.opts() == best and ms > 0
    say("best", best, ms)
    b.run()
    check_batch(b, qs, refs, f"tuned {best}")
    assert b.time(reps=3) > 0
    b.free()


def test_batch_view_orphaned_by_free(ctx):
    qs, hs, refs = c5_setup(ctx, 3, 20_000, 1000, 20_000, seed=dg.MASTER_SEED + 58)
    b = hawk.Batch(ctx, hs)
    b.run()
    r = b.result(0)
    r.info()
    b.free()
    with pytest.raises(hawk.HawkError):
        r.info()
    r.free()


def feasible_variants(ctx, h, rng, k):
    """k variants drawn from the query's space that execute on their own
    (a local table that cannot fit in LDS is infeasible for large group counts)."""
    space = hawk.variant_space(h)
    out = []
    for i in rng.permutation(len(space)):
        v = space[i]
        try:
            hawk.execute(ctx, h, v).free()
        except hawk.HawkError as e:
            if e.code == hawk.HAWK_E_INFEASIBLE:
                continue
            raise
        out.append(v)
        if len(out) == k:
            break
    return out


def test_batch_per_query_variants(ctx):
    """Every query in a variant of its own space (or in the tile kernels),
    all in one graph: each result against the oracle over replays, after a
    re-capture for another schedule, and with the same variants given again."""
    say("batch: per-query variants")
    qs, hs, refs = c5_setup(ctx, 18, 1_000_000, 1000, 1_000_000, seed=dg.MASTER_SEED + 60)
    rng = np.random.default_rng(3)
    variants = []
    for n, h in enumerate(hs):
        variants.append(hawk.TILE if n % 4 == 3 else feasible_variants(ctx, h, rng, 1)[0])
    for q, v in zip(qs, variants):
        say("kind", q["kind"], "rows", q["rows"], "tile" if v.thread_mult == 0 else hawk.format_variant(v))
    b = hawk.Batch(ctx, hs, variants=variants, tile_rows_log2=15, wgs_per_cu=4, order=0)
    for rep in range(2):
        b.run()
        check_batch(b, qs, refs, f"per-query variants, replay {rep}")
    assert b.time(reps=2) > 0
    best, _ = b.autotune(reps=1)
    b.run()
    check_batch(b, qs, refs, f"per-query variants, schedule {best}")
    b.free()
    # variants that the tile kernels do not have: cuckoo tables, global
    # aggregation, sequential access, single-pass projection
    special = []
    for q, h in zip(qs, hs):
        if q["kind"] == 1:
            special.append(hawk.variant(proj_strategy=0, mem=0, pred=1))
        else:
            special.append(hawk.variant(agg_strategy=1, ht=1, hash=1, mem=0, pred=1, wg_size=512))
    b = hawk.Batch(ctx, hs, variants=special)
    b.run()
    b.run()
    check_batch(b, qs, refs, "cuckoo/global/sequential/single-pass")
    b.free()


def test_batch_cross_join_queries(ctx):
    """Pipelines with a CROSS_JOIN in a batch, in the tile kernels and in
    variants of their own, next to ordinary ones."""
    say("batch: cross joins")
    qs, hs, refs = c5_setup(ctx, 4, 200_000, 1000, 200_000, seed=dg.MASTER_SEED + 61)
    specs = [q["spec"] for q in qs]
    for sink in ("project", "group"):
        tables, spec = dg.cross_join(n=9_000, m=40, sink=sink)
        tables = {f"bx{sink}_{t}": c for t, c in tables.items()}
        spec["main"]["table"], spec["main"]["cross"] = f"bx{sink}_t", f"bx{sink}_u"
        spec["builds"][0]["table"] = f"bx{sink}_d"
        refs.append(oracle.run(tables, spec))
        ctx.register_numpy(tables)
        hs.append(hawk.build_query(ctx, spec))
        specs.append(spec)
    fake = [{"spec": s, "kind": 0, "rows": 0} for s in specs]
    for variants in (None, [hawk.TILE] * 4 + [hawk.variant(proj_strategy=0, mem=1),
                                              hawk.variant(agg_strategy=1, ht=1, hash=1, wg_size=256)]):
        b = hawk.Batch(ctx, hs, variants=variants, tile_rows_log2=14, wgs_per_cu=2)
        b.run()
        b.run()
        check_batch(b, fake, refs, "cross joins" if variants is None else "cross joins, own variants")
        b.free()


def test_batch_per_query_variants_run_time_kernels(ctx):
    """Per-query variants in one graph with run-time compiled kernels: star
    joins on one 1024-thread workgroup per CU (their first join table copied
    into LDS), aggregations and projections in variants of their own; every
    result against the oracle over two replays."""
    say("batch: per-query variants, run-time kernels")
    ctx.set_jit(True)
    qs, hs, refs = c5_setup(ctx, 12, 1_000_000, 1000, 1_000_000, seed=dg.MASTER_SEED + 62)
    assert 3 in {q["kind"] for q in qs}
    variants = []
    for q in qs:
        if q["kind"] == 3:
            variants.append(hawk.variant(agg_strategy=0, ht=0, hash=1, mem=1, pred=0, thread_mult=1, wg_size=1024))
        elif q["kind"] == 2:
            variants.append(hawk.variant(agg_strategy=0, ht=0, hash=1, mem=1, pred=1, thread_mult=1, wg_size=1024))
        else:
            variants.append(hawk.variant(proj_strategy=1, mem=1, pred=0, thread_mult=1024, wg_size=256))
    b = hawk.Batch(ctx, hs, variants=variants, tile_rows_log2=15, wgs_per_cu=4, order=0)
    for rep in range(2):
        b.run()
        check_batch(b, qs, refs, f"run-time kernels, replay {rep}")
    b.free()
    assert ctx.jit_stats()[0] >= 2
