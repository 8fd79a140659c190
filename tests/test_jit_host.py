"""The kernels generated for run-time compilation compile (hipRTC, gfx950)
without a device: for every benchmark pipeline in its timed variant and in
variants that switch on the other generated code paths (predication,
Murmur hashing, spilling, probes, the SIMD filter and unrolling). A source
that fails to compile would otherwise show only on a GPU, at its first
execution."""
import pytest

from paper_1709_00700_amd import hawk

import bench


@pytest.fixture(scope="module")
def plan_ctx():
    c = hawk.PlanningContext()
    yield c
    _QUERIES.clear()
    c.close()


_QUERIES = {}


def query_of(ctx, name):
    if name in _QUERIES:
        return _QUERIES[name]
    tables, spec = bench.make_pipeline(name, rows=4096)
    # the full workload's row counts (spilling depends on them)
    full = {"c1": 1_000_000, "c1_256m": 256 << 20, "c2u": 64 << 20, "c2z": 64 << 20, "c3": 120_000_000,
            "c4": 600_000_000}[name]
    main = spec["main"]["table"]
    shapes = {t: {c: (a.dtype, full if t == main else len(a)) for c, a in cols.items()} for t, cols in tables.items()}
    ctx.register_shapes(shapes)
    _QUERIES[name] = hawk.build_query(ctx, spec)
    return _QUERIES[name]


CASES = [(w, {}) for w in ("c1", "c1_256m", "c2u", "c2z", "c3", "c4")] + [
    ("c2u", {"pred": 0, "hash": 0}),
    ("c2z", {"pred": 1}),
    ("c3", {"pred": 1, "hash": 0}),
    ("c4", {"pred": 0, "thread_mult": 1, "wg_size": 1024}),
    ("c1", {"filter_mode": 1, "thread_mult": 65536}),
    ("c1", {"unroll": 2, "pred": 1}),
]


@pytest.mark.parametrize("name,kw", CASES, ids=[f"{w}-{i}" for i, (w, _) in enumerate(CASES)])
def test_generated_kernels_compile(plan_ctx, name, kw):
    q = query_of(plan_ctx, name)
    v = hawk.variant(**dict(bench.DEFAULT_VARIANTS[name], **kw))
    hawk.jit_compile_check(plan_ctx, q, v)
    # the context's own setting is left as it was: nothing was kept
    assert plan_ctx.jit_stats()[0] == 0


def test_compile_check_reports_bad_arguments(plan_ctx):
    q = query_of(plan_ctx, "c2u")
    assert hawk.L().hawk_jit_compile_check(plan_ctx.handle, q.handle, None) == hawk.HAWK_E_ARG
    assert hawk.L().hawk_jit_compile_check(None, q.handle, None) == hawk.HAWK_E_ARG


def _generated_sources(ctx, q, v, tmp_path, monkeypatch):
    d = tmp_path / "gen"
    d.mkdir(parents=True)
    monkeypatch.setenv("HAWK_JIT_DUMP", str(d))
    hawk.jit_compile_check(ctx, q, v)
    return [p.read_text() for p in sorted(d.glob("*.hip"))]


def test_small_join_table_staged_in_lds(plan_ctx, tmp_path, monkeypatch):
    # the star join's first dimension (2.5k rows: 8192 slots, 64 KiB) fits
    # half of a whole-CU workgroup's LDS and is copied there; the others
    # (0.5-4 MB) are probed in device memory
    q = query_of(plan_ctx, "c3")
    v = hawk.variant(**dict(bench.DEFAULT_VARIANTS["c3"], thread_mult=1, wg_size=1024))
    (src,) = _generated_sources(plan_ctx, q, v, tmp_path, monkeypatch)
    assert "stage_join(P.probes[0].t, lds + " in src and ", 13u);" in src
    assert "stage_join(P.probes[1]" not in src and "stage_join(P.probes[3]" not in src
    assert "__syncthreads();" in src


def test_no_staging_where_the_table_would_cost_residency(plan_ctx, tmp_path, monkeypatch):
    # eight workgroups per CU keep two local tables per CU: the 64 KiB
    # table does not fit beside one
    q = query_of(plan_ctx, "c3")
    v = hawk.variant(**dict(bench.DEFAULT_VARIANTS["c3"], thread_mult=8, wg_size=512))
    (src,) = _generated_sources(plan_ctx, q, v, tmp_path, monkeypatch)
    assert "stage_join" not in src


def test_scalar_aggregate_kernel_generated(plan_ctx, tmp_path, monkeypatch):
    # AGGREGATE without grouping attributes: its run-time kernel is
    # generated and compiles, in both aggregation strategies
    from paper_1709_00700_amd import datagen as dg
    tables, spec = dg.c4_wide(n=4096)
    spec["main"]["group_by"] = []
    spec["main"].pop("groups_hint", None)
    tables = {"scalar_t": tables["t"]}
    spec["main"]["table"] = "scalar_t"
    plan_ctx.register_shapes({t: {c: (a.dtype, len(a)) for c, a in cols.items()} for t, cols in tables.items()})
    q = hawk.build_query(plan_ctx, spec)
    for strat in (0, 1):
        v = hawk.variant(mem=1, pred=strat, ht=0, hash=1, agg_strategy=strat, thread_mult=4, wg_size=256)
        (src,) = _generated_sources(plan_ctx, q, v, tmp_path / f"s{strat}", monkeypatch)
        assert "hk_jit_scalar" in src and "scalar_body<" in src


def test_staging_keeps_small_global_workgroups_resident(plan_ctx, tmp_path, monkeypatch):
    # the global strategy has no local table: with 64-thread workgroups the
    # 64 KiB table would leave two waves per CU, so it stays in device memory
    q = query_of(plan_ctx, "c3")
    v = hawk.variant(**dict(bench.DEFAULT_VARIANTS["c3"], agg_strategy=1, wg_size=64))
    (src,) = _generated_sources(plan_ctx, q, v, tmp_path, monkeypatch)
    assert "stage_join" not in src
