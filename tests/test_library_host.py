"""Host-side checks of libhawk.so that need no GPU: exported symbols, plan
validation, the variant space of Section 9.2, features, and Algorithm 1
against its oracle under fake timing backends."""
import ctypes
import itertools
import math
import os
import re

import numpy as np
import pytest

from oracle import alg1
from paper_1709_00700_amd import datagen as dg
from paper_1709_00700_amd import hawk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "hawk.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hawk_[a-z_0-9]+)\s*\(", txt)) - {"hawk_cost_fn"})


def test_library_exports_every_declared_symbol():
    lib = hawk.L()
    declared = header_functions()
    assert declared, "no declarations parsed"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(hawk.EXPORTS) == declared


def test_device_context_fails_cleanly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import ctypes
    h = ctypes.c_void_p()
    assert hawk.L().hawk_ctx_create(0, None, ctypes.byref(h)) == hawk.HAWK_E_DEVICE


@pytest.fixture
def plan_ctx():
    c = hawk.PlanningContext()
    yield c
    c.close()


def _shapes(tables):
    return {t: {c: a[:1] if len(a) else a for c, a in cols.items()} for t, cols in tables.items()}


@pytest.mark.parametrize("name,expected", [("c1", 32), ("c2u", 896), ("c2z", 896), ("c3", 896), ("c4", 896)])
def test_variant_space_sizes(plan_ctx, name, expected):
    tables, spec = dg.workload(name, n=10) if name != "c3" else dg.c3_star_join(n=10, dims=(5, 5, 5, 5))
    plan_ctx.register_shapes(tables)
    q = hawk.build_query(plan_ctx, spec)
    vs = hawk.variant_space(q)
    assert len(vs) == expected
    assert len({hawk.format_variant(v) for v in vs}) == expected   # all distinct
    # the first variant takes the first value of every dimension (Algorithm 1, line 1 reading)
    v0 = vs[0].as_dict()
    if q.kind == 1:
        assert (v0["proj_strategy"], v0["mem"], v0["pred"]) == (0, 0, 0)
    else:
        assert (v0["agg_strategy"], v0["mem"], v0["pred"], v0["ht"], v0["hash"], v0["thread_mult"],
                v0["wg_size"]) == (0, 0, 0, 0, 0, 1, 16)


def test_variant_space_counts_by_dimension(plan_ctx):
    tables, spec = dg.workload("c2u", n=10)
    plan_ctx.register_shapes(tables)
    vs = [v.as_dict() for v in hawk.variant_space(hawk.build_query(plan_ctx, spec))]
    local = [v for v in vs if v["agg_strategy"] == 0]
    glob = [v for v in vs if v["agg_strategy"] == 1]
    assert len(local) == 2 * 2 * 2 * 2 * 7 * 7 and len(glob) == 2 * 2 * 2 * 2 * 7
    assert sorted({v["thread_mult"] for v in local}) == [1, 8, 64, 256, 1024, 16384, 65536]
    assert sorted({v["wg_size"] for v in vs}) == [16, 32, 64, 128, 256, 512, 1024]
    # non-grouped aggregation without joins has no hash-table dimensions
    spec2 = dict(spec)
    spec2["main"] = dict(spec["main"], group_by=[])
    assert len(hawk.variant_space(hawk.build_query(plan_ctx, spec2))) == 2 * 2 * (49 + 7)


def test_projection_with_probe_has_table_dims(plan_ctx):
    tables = {"d": {"k": np.zeros(4, np.int32), "g": np.zeros(4, np.int32)},
              "f": {"fk": np.zeros(4, np.int32), "v": np.zeros(4, np.int64)}}
    plan_ctx.register_shapes(tables)
    spec = {"builds": [{"table": "d", "filters": [], "key": "k", "payload": "g"}],
            "main": {"table": "f", "filters": [], "probes": [("fk", 0, "p")], "arith": [], "project": ["v", "p"]}}
    assert len(hawk.variant_space(hawk.build_query(plan_ctx, spec))) == 32 * 4


def _expect(plan_ctx, spec, code):
    with pytest.raises(hawk.HawkError) as e:
        hawk.build_query(plan_ctx, spec)
    assert e.value.code == code, e.value


def test_plan_validation_errors(plan_ctx):
    tables = {"t": {"a": np.zeros(3, np.int32), "w": np.zeros(3, np.int64)},
              "d": {"k": np.zeros(3, np.int32), "big": np.zeros(3, np.int64)}}
    plan_ctx.register_shapes(tables)
    base = {"table": "t", "filters": [], "probes": [], "arith": []}
    _expect(plan_ctx, {"builds": [], "main": dict(base, project=["nope"])}, hawk.HAWK_E_NOTFOUND)
    _expect(plan_ctx, {"builds": [], "main": dict(base, filters=[("zz", 0, 1)], project=["a"])}, hawk.HAWK_E_NOTFOUND)
    _expect(plan_ctx, {"builds": [], "main": dict(base, group_by=["w"], aggs=[("count", None, False)])},
            hawk.HAWK_E_TYPE)
    _expect(plan_ctx, {"builds": [{"table": "d", "filters": [], "key": "big", "payload": "k"}],
                       "main": dict(base, probes=[("a", 0, "p")], project=["p"])}, hawk.HAWK_E_TYPE)
    _expect(plan_ctx, {"builds": [], "main": dict(base, probes=[("a", 0, "p")], project=["p"])}, hawk.HAWK_E_PLAN)
    _expect(plan_ctx, {"builds": [], "main": dict(base, group_by=["a"], aggs=[("count", None, False)] * 9)},
            hawk.HAWK_E_PLAN)
    many = [(f"x{i}", "add", "a", 1) for i in range(8)] + [(f"y{i}", "add", "a", 1) for i in range(8)]
    _expect(plan_ctx, {"builds": [], "main": dict(base, arith=many, project=["a"])}, hawk.HAWK_E_PLAN)
    _expect(plan_ctx, {"builds": [], "main": dict(base, arith=[("a", "add", "a", 1)], project=["a"])},
            hawk.HAWK_E_PLAN)
    # a valid plan compiles; executing on the planning context is refused
    q = hawk.build_query(plan_ctx, {"builds": [], "main": dict(base, project=["a"])})
    with pytest.raises(hawk.HawkError) as e:
        hawk.execute(plan_ctx, q, hawk.variant())
    assert e.value.code == hawk.HAWK_E_DEVICE


@pytest.mark.parametrize("dtype,addr,ok", [(1, 0x1001, True), (2, 0x1002, False), (2, 0x1004, True),
                                           (3, 0x1004, False), (3, 0x1008, True)])
def test_columns_must_be_aligned_to_their_element_size(plan_ctx, dtype, addr, ok):
    col = (hawk.hawk_column * 1)(hawk.hawk_column(b"c", dtype, 0, ctypes.c_void_p(addr)))
    tid = ctypes.c_int32()
    st = hawk.L().hawk_table_register(plan_ctx.handle, f"t{dtype}_{addr}".encode(), 10, col, 1, ctypes.byref(tid))
    assert (st == hawk.HAWK_OK) == ok
    if not ok:
        assert st == hawk.HAWK_E_ARG


def test_features_follow_their_definition(plan_ctx):
    tables, spec = dg.c4_wide(n=10)
    plan_ctx.register_shapes({"t": {c: (a.dtype, 600_000_000) for c, a in tables["t"].items()}})
    q = hawk.build_query(plan_ctx, spec)
    q.set_stats(0.25)
    v = hawk.variant(agg_strategy=0, mem=1, pred=1, ht=1, hash=0, thread_mult=8, wg_size=512)
    f = q.features(v)
    assert f[0] == pytest.approx(math.log2(600_000_001))
    assert f[1] == pytest.approx(0.25)
    assert f[2] == pytest.approx(math.log2(7))
    assert f[3] == 1 + 1 + 4 + 8 + 4 + 4          # flag1, flag2, qty, price, disc, tax
    assert f[4] == 0
    assert f[5] == 8 * (2 + 5 + 1 + 1 + 1)           # key, count, 4 narrow + 1 wide sum, min, max, avg sum
    assert f[6] == 0 and f[7] == pytest.approx(math.log2(8 * 256 * 512)) and f[8] == 9
    assert (f[9], f[10], f[11]) == (1, 1, 2)


# ------------------------------------------------------------------ Algorithm 1 with fake timers
def lib_alg1(sizes, cost, q=5, order=None):
    return hawk.learn_feature_wise(sizes, cost, q=q, order=order)


def test_alg1_separable_finds_optimum_in_one_sweep():
    rng = np.random.default_rng(3)
    sizes = [2, 7, 7, 2, 2, 2, 2]
    tabs = [rng.uniform(1, 10, s) for s in sizes]
    calls = []

    def cost(cfg):
        calls.append(cfg)
        return sum(t[c] for t, c in zip(tabs, cfg))

    cfg, n = lib_alg1(sizes, cost)
    assert cfg == tuple(int(np.argmin(t)) for t in tabs)
    # exhaustive search agrees for a separable cost
    best = min(itertools.product(*[range(s) for s in sizes]), key=cost)
    assert cfg == best
    # sweep 1 reaches the optimum and sweep 2 only confirms it: at most two sweeps
    assert n <= 1 + 2 * sum(s - 1 for s in sizes)
    assert (cfg, n) == alg1.learn_feature_wise(sizes, cost)


def test_alg1_ties_keep_first_value_and_infeasible_is_never_chosen():
    cfg, n = lib_alg1([3, 4, 5], lambda c: 1.0)
    assert cfg == (0, 0, 0)
    inf_first = lambda c: math.inf if c[0] == 0 else float(c[0] + c[1])
    cfg, _ = lib_alg1([3, 3], inf_first)
    assert cfg == (1, 0)
    cfg, _ = lib_alg1([2, 2], lambda c: math.inf)   # nothing feasible: stays at the start
    assert cfg == (0, 0)


@pytest.mark.parametrize("seed", range(20))
def test_alg1_matches_oracle_on_random_tables(seed):
    rng = np.random.default_rng(seed)
    sizes = list(rng.integers(1, 6, size=int(rng.integers(1, 6))))
    table = rng.uniform(0, 100, size=sizes)
    table[rng.random(size=sizes) < 0.1] = math.inf
    cost = lambda c: float(table[c])
    q = int(rng.integers(1, 6))
    order = list(rng.permutation(len(sizes))) if seed % 2 else None
    got = lib_alg1([int(s) for s in sizes], cost, q=q, order=order)
    exp = alg1.learn_feature_wise([int(s) for s in sizes], cost, q=q, order=order)
    assert got == exp
    cfg, n = got
    assert n <= q * sum(sizes) + 1


@pytest.mark.parametrize("seed", range(10))
def test_alg1_fixed_point_is_coordinatewise_optimal(seed):
    rng = np.random.default_rng(50 + seed)
    sizes = [3, 4, 3, 2]
    table = rng.uniform(0, 10, size=sizes)
    cost = lambda c: float(table[c])
    cfg, _ = lib_alg1(sizes, cost, q=50)
    for i, s in enumerate(sizes):
        for d in range(s):
            w = list(cfg)
            w[i] = d
            assert table[tuple(w)] >= table[cfg]


def test_handles_outliving_their_context_are_orphaned():
    import ctypes
    c = hawk.PlanningContext()
    tables, spec = dg.workload("c2u", n=10)
    c.register_shapes(tables)
    q = hawk.build_query(c, spec)
    c.close()                      # the query's context is gone
    f = (ctypes.c_float * 12)()
    assert hawk.L().hawk_features(q.handle, ctypes.byref(hawk.variant()), f) == hawk.HAWK_E_ARG
    hawk.L().hawk_query_free(q.handle)   # only host memory is released; no crash
    q.handle = None


@pytest.mark.parametrize("mode", [hawk.HAWK_EXPLORE_EXHAUSTIVE, hawk.HAWK_EXPLORE_FEATURE_WISE])
def test_explore_resumes_from_timing_log(plan_ctx, tmp_path, mode):
    """A planning context cannot time anything: the first exploration logs its
    workload line and stops with HAWK_E_DEVICE. Once the log holds a timing for
    every variant of that workload, a resumed exploration measures nothing and
    returns the argmin of the logged times (ties: the first in search order)."""
    tables, spec = dg.c2_aggregation(n=10, dist="uniform")
    plan_ctx.register_shapes(_shapes(tables))
    q = hawk.build_query(plan_ctx, spec)
    db = str(tmp_path / "timings.tsv")
    with pytest.raises(hawk.HawkError) as e:
        hawk.explore(plan_ctx, [q], mode, timing_db=db)
    assert e.value.code == hawk.HAWK_E_DEVICE
    head = [ln for ln in open(db) if ln.startswith("#workload")]
    assert len(head) == 1
    sig = head[0].split("\t")[1]
    space = hawk.variant_space(q)
    rng = np.random.default_rng(3)
    times = {hawk.format_variant(v): float(rng.uniform(1.0, 9.0)) for v in space}
    pruned = [hawk.format_variant(v) for v in space[::7]]
    with open(db, "a") as f:
        f.write("other\t0" + "\t0" * 12 + f"\t{hawk.format_variant(space[0])}\t0.001\t0\n")  # another workload
        for key, ms in times.items():
            st = hawk.HAWK_E_TIMEOUT if key in pruned else 0
            f.write(f"{sig}\t0" + "\t0" * 12 + f"\t{key}\t{-1.0 if st else ms:.6f}\t{st}\n")
    best, rep = hawk.explore(plan_ctx, [q], mode, timing_db=db, resume=True)
    assert rep["evaluated"] == 0 and rep["reused"] == len(space)
    feasible = {k: t for k, t in times.items() if k not in pruned}
    if mode == hawk.HAWK_EXPLORE_EXHAUSTIVE:
        assert hawk.format_variant(best) == min(feasible, key=feasible.get)
    assert rep["best_ms"] == pytest.approx(feasible[hawk.format_variant(best)], abs=1e-6)


def test_noalloc_sizing_on_a_planning_context(plan_ctx):
    """hawk_execute_noalloc's sizing call (no result columns) needs no device:
    a projection needs its input rows plus the dump slot, a grouped
    aggregation the slots of its table (a power of two >= 2 x the group hint,
    at least 64) plus the side slot, a non-grouped one a single row; asking
    to run on a planning context is a device error."""
    tables, spec = dg.c1_projection(n=1000)
    plan_ctx.register_shapes({"p_" + t: c for t, c in tables.items()})
    spec["main"]["table"] = "p_t"
    q = hawk.build_query(plan_ctx, spec)
    assert hawk.execute_noalloc(plan_ctx, q, hawk.variant(proj_strategy=1, thread_mult=64)) == 1001
    assert hawk.execute_noalloc(plan_ctx, q, hawk.variant(proj_strategy=0)) == 1001
    tables, spec = dg.c3_star_join(n=500, dims=(40, 40, 40, 40))
    plan_ctx.register_shapes({"s_" + t: c for t, c in tables.items()})
    spec["main"]["table"] = "s_f"
    for b in spec["builds"]:
        b["table"] = "s_" + b["table"]
    q = hawk.build_query(plan_ctx, spec)
    hint = spec["main"]["groups_hint"]
    slots = max(64, 1 << (2 * hint - 1).bit_length())
    assert hawk.execute_noalloc(plan_ctx, q, hawk.variant(agg_strategy=0, thread_mult=8, wg_size=256)) == slots + 1
    spec["main"]["group_by"] = []
    q = hawk.build_query(plan_ctx, spec)
    assert hawk.execute_noalloc(plan_ctx, q, hawk.variant(agg_strategy=1, wg_size=256)) == 1
    with pytest.raises(hawk.HawkError) as e:
        hawk.execute_noalloc(plan_ctx, q, hawk.variant(), [0x1000] * 3, 1)
    assert e.value.code == hawk.HAWK_E_DEVICE


def test_cross_join_plan_validation(plan_ctx):
    """CROSS_JOIN (Table 1): the pipeline loops over the product of its table
    and a second one; names must differ between the two, the product must
    stay below 2^32 pairs, and its variant space is that of its sink."""
    tables, spec = dg.cross_join(n=100, m=7, sink="project")
    plan_ctx.register_shapes({"cj_" + t: c for t, c in tables.items()})
    spec["main"]["table"], spec["main"]["cross"] = "cj_t", "cj_u"
    spec["builds"][0]["table"] = "cj_d"
    q = hawk.build_query(plan_ctx, spec)
    assert len(hawk.variant_space(q)) == 32 * 4   # projection with a probe: hash-table dimensions too
    assert hawk.execute_noalloc(plan_ctx, q, hawk.variant(proj_strategy=1, thread_mult=8)) == 100 * 7 + 1
    bad = {**spec, "main": {**spec["main"], "cross": "cj_t"}}
    _expect(plan_ctx, bad, hawk.HAWK_E_PLAN)                       # every name in both tables
    plan_ctx.register_shapes({"cj_big": {"a": ("int32", 1 << 20), "v": ("int64", 1 << 20)},
                              "cj_wide": {"b": ("int32", 1 << 12), "fk": ("int32", 1 << 12), "w": ("int8", 1 << 12)}})
    big = {**spec, "main": {**spec["main"], "table": "cj_big", "cross": "cj_wide"}}
    _expect(plan_ctx, big, hawk.HAWK_E_PLAN)                       # 2^32 pairs


def test_cross_join_quotient_by_reciprocal():
    """The device divides a pipeline row v < 2^32 by the second table's row
    count d as the high word of (2^64 / d rounded up) * v: exact for every
    32-bit v and d > 1 (the identity the kernels rely on)."""
    rng = np.random.default_rng(11)
    ds = [2, 3, 7, 64, 1000, 65537, (1 << 31) - 1, (1 << 32) - 1] + [int(x) for x in rng.integers(2, 1 << 32, 40)]
    vs = [0, 1, (1 << 32) - 1, (1 << 31)] + [int(x) for x in rng.integers(0, 1 << 32, 200)]
    for d in ds:
        m = (2 ** 64 - 1) // d + 1
        for v in vs + [d - 1, d, d + 1, 2 * d - 1]:
            if v < 1 << 32:
                assert (m * v) >> 64 == v // d, (d, v)


def test_extra_variant_dimensions(plan_ctx):
    """Extra dimensions (hawk_ctx_set_variant_dims) multiply in where they
    apply: unrolling (2, 1) and the SIMD filter for multi-pass coalesced
    projections (the filter only without probes), robin hood as a third
    table kind for pipelines with probes; features code them ordinally."""
    tables, c1 = dg.c1_projection(n=10)
    plan_ctx.register_shapes({"xd_t": tables["t"]})
    c1["main"]["table"] = "xd_t"
    tables, c3 = dg.c3_star_join(n=10, dims=(5, 5, 5, 5))
    plan_ctx.register_shapes({"xd_" + t: c for t, c in tables.items()})
    c3["main"]["table"] = "xd_f"
    for b in c3["builds"]:
        b["table"] = "xd_" + b["table"]
    proj_probe = {"builds": c3["builds"][:1],
                  "main": {"table": "xd_f", "filters": [], "probes": [("fk0", 0, "p")], "arith": [], "project": ["p"]}}
    q1, q3, qp = (hawk.build_query(plan_ctx, s) for s in (c1, c3, proj_probe))
    assert [len(hawk.variant_space(q)) for q in (q1, q3, qp)] == [32, 896, 128]
    plan_ctx.set_variant_dims(hawk.HAWK_DIM_UNROLL)
    assert len(hawk.variant_space(q1)) == 4 + 14 + 14 * 3
    plan_ctx.set_variant_dims(hawk.HAWK_DIM_UNROLL | hawk.HAWK_DIM_SIMD_FILTER)
    vs = hawk.variant_space(q1)
    assert len(vs) == 4 + 14 + 14 * 4
    simd = [v for v in vs if v.filter_mode]
    assert len(simd) == 14 and all(v.mem == 1 and v.proj_strategy == 1 for v in simd)
    assert "filter=simd" in hawk.format_variant(simd[0])
    assert q1.features(simd[0])[9] == simd[0].pred + 2
    u1 = next(v for v in vs if v.unroll == 1)
    assert q1.features(u1)[10] == 1 + 2 * 2 and "unroll=1" in hawk.format_variant(u1)
    plan_ctx.set_variant_dims(hawk.HAWK_DIM_ROBIN_HOOD | hawk.HAWK_DIM_SIMD_FILTER)
    assert len(hawk.variant_space(q3)) == 896 // 4 * 6       # three table kinds with probes
    vp = hawk.variant_space(qp)
    assert len(vp) == 128 // 4 * 6                          # no SIMD filter with probes
    robin = next(v for v in vp if v.ht == hawk.HAWK_ROBIN_HOOD)
    assert "ht=robin" in hawk.format_variant(robin) and qp.features(robin)[11] == 2 * 2 + robin.hash
    assert len(hawk.variant_space(q1)) == 32 + 14             # no table: no robin hood
    plan_ctx.set_variant_dims(0)
    assert [len(hawk.variant_space(q)) for q in (q1, q3, qp)] == [32, 896, 128]
    with pytest.raises(hawk.HawkError):
        plan_ctx.set_variant_dims(64)
