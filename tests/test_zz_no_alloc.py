"""GPU check of hawk_execute_noalloc, the execution whose buffers all lie in
the library's per-device scratch array (plus the caller's result columns):
through the C ABI, its results equal hawk_execute's for the same query and
variant, element by element (AVG within 1e-12 relative), on two calls in a
row where the second runs a smaller input over the scratch the first one
left behind."""
import ctypes

import numpy as np
import pytest

from gpu_common import compare, say
from paper_1709_00700_amd import datagen as dg
from paper_1709_00700_amd import hawk

pytestmark = pytest.mark.gpu

ESIZE = {hawk.HAWK_RES_I64: 8, hawk.HAWK_RES_I128: 16, hawk.HAWK_RES_F64: 8}


@pytest.fixture
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hawk.Context(0)
    yield c
    c.close()


def column_kinds(res: hawk.Result) -> list:
    _, ncols = res.info()
    kinds = []
    for c in range(ncols):
        k, p = ctypes.c_int32(), ctypes.c_void_p()
        hawk.check(hawk.L().hawk_result_column(res.handle, c, ctypes.byref(k), ctypes.byref(p)), res.ctx.handle)
        kinds.append(k.value)
    return kinds


def run_noalloc(ctx, q, v, spec, kinds):
    """Sizing call, then the execution into torch-allocated result columns;
    returns the result in the layout of Result.to_numpy."""
    import torch
    cap = hawk.execute_noalloc(ctx, q, v)
    assert cap >= 1
    bufs = [torch.empty(cap * ESIZE[k], dtype=torch.uint8, device="cuda") for k in kinds]
    n = hawk.execute_noalloc(ctx, q, v, [b.data_ptr() for b in bufs], cap)
    torch.cuda.synchronize()
    cols = []
    for k, b in zip(kinds, bufs):
        raw = b[: n * ESIZE[k]].cpu().numpy()
        if k == hawk.HAWK_RES_I128:
            lo, hi = raw.view(np.uint64)[0::2], raw.view(np.int64)[1::2]
            cols.append(np.array([(int(h) << 64) | int(l) for l, h in zip(lo, hi)], dtype=object))
        elif k == hawk.HAWK_RES_F64:
            cols.append(raw.view(np.float64).copy())
        else:
            cols.append(raw.view(np.int64).copy())
    m = spec["main"]
    if "project" in m:
        return {"kind": "project", "rows": n, "cols": cols}
    ng = len(m.get("group_by", []))
    keys, aggs, cnt = cols[:ng], cols[ng:-1], cols[-1]
    order = np.lexsort(tuple(reversed(keys))) if ng else np.arange(n)
    return {"kind": "aggregate", "rows": n, "keys": [k[order] for k in keys], "count": cnt[order],
            "aggs": [a[order] for a in aggs]}


def check_pair(ctx, make, sizes, v, label):
    """Two calls in a row, the second on the smaller input, each against hawk_execute."""
    for i, n in enumerate(sizes):
        tables, spec = make(n)
        ren = {t: f"{label}{i}_{t}" for t in tables}
        tables = {ren[t]: c for t, c in tables.items()}
        spec["main"]["table"] = ren[spec["main"]["table"]]
        if spec["main"].get("cross"):
            spec["main"]["cross"] = ren[spec["main"]["cross"]]
        for b in spec["builds"]:
            b["table"] = ren[b["table"]]
        ctx.register_numpy(tables)
        q = hawk.build_query(ctx, spec)
        say(label, "rows", n, hawk.format_variant(v))
        r = hawk.execute(ctx, q, v)
        ref = r.to_numpy(spec)
        kinds = column_kinds(r)
        r.free()
        got = run_noalloc(ctx, q, v, spec, kinds)
        compare(got, ref, spec, f"{label} n={n}")
        say(label, "rows", n, "result rows", ref["rows"], "ok")


def test_projection_multi_and_single_pass(ctx):
    for k, v in enumerate((hawk.variant(proj_strategy=1, mem=1, pred=0, thread_mult=1024),
                           hawk.variant(proj_strategy=1, mem=0, pred=1, thread_mult=64),
                           hawk.variant(proj_strategy=0, mem=1, pred=0))):
        check_pair(ctx, lambda n: dg.c1_projection(n=n), [1_000_000, 100_003], v, f"proj{k}_")


def test_grouped_aggregation_local_and_global(ctx):
    make = lambda n: dg.c2_aggregation(n=n, dist="zipf", nranks=3000)  # noqa: E731
    for k, v in enumerate((hawk.variant(agg_strategy=0, ht=0, hash=1, thread_mult=8, wg_size=256),
                           hawk.variant(agg_strategy=1, ht=1, hash=0, wg_size=512),
                           hawk.variant(agg_strategy=0, ht=1, hash=0, pred=1, thread_mult=1, wg_size=1024))):
        check_pair(ctx, make, [2_000_000, 300_001], v, f"agg{k}_")


def test_star_join_and_wide_sums(ctx):
    check_pair(ctx, lambda n: dg.c3_star_join(n=n), [1_500_000, 200_000],
               hawk.variant(agg_strategy=0, ht=0, hash=1, thread_mult=8, wg_size=512), "star")
    check_pair(ctx, lambda n: dg.c4_wide(n=n, price_hi=1 << 40), [1_000_000, 99_999],
               hawk.variant(agg_strategy=0, ht=0, hash=1, pred=1, thread_mult=8, wg_size=512), "wide")


def test_limits_are_reported(ctx):
    import torch
    # a spilling aggregation needs more scratch than the array holds
    tables, spec = dg.c2_aggregation(n=8_000_000, dist="zipf", nranks=1_000_000)
    tables = {"lim_t": tables["t"]}
    spec["main"]["table"] = "lim_t"
    ctx.register_numpy(tables)
    q = hawk.build_query(ctx, spec)
    v = hawk.variant(agg_strategy=0, ht=0, hash=1, thread_mult=1, wg_size=1024)
    cap = hawk.execute_noalloc(ctx, q, v)
    bufs = [torch.empty(cap * 8, dtype=torch.uint8, device="cuda") for _ in range(6)]
    with pytest.raises(hawk.HawkError) as e:
        hawk.execute_noalloc(ctx, q, v, [b.data_ptr() for b in bufs], cap)
    assert e.value.code == hawk.HAWK_E_CAPACITY
    # result columns smaller than the need, and a wrong column count
    tables, spec = dg.c2_aggregation(n=100_000, dist="uniform")
    tables = {"lim_u": tables["t"]}
    spec["main"]["table"] = "lim_u"
    ctx.register_numpy(tables)
    q = hawk.build_query(ctx, spec)
    v = hawk.variant(agg_strategy=1, ht=0, hash=0, wg_size=256)
    cap = hawk.execute_noalloc(ctx, q, v)
    with pytest.raises(hawk.HawkError) as e:
        hawk.execute_noalloc(ctx, q, v, [b.data_ptr() for b in bufs], cap - 1)
    assert e.value.code == hawk.HAWK_E_ARG
    with pytest.raises(hawk.HawkError) as e:
        hawk.execute_noalloc(ctx, q, v, [b.data_ptr() for b in bufs[:5]], cap)
    assert e.value.code == hawk.HAWK_E_ARG
    # the entry point still works after the errors
    n = hawk.execute_noalloc(ctx, q, v, [b.data_ptr() for b in bufs[:6]], cap)
    assert n == 16


def test_cross_join(ctx):
    # global table (a local one too small for the groups would spill, which
    # needs scratch for every pair)
    check_pair(ctx, lambda n: dg.cross_join(n=n, m=48, sink="group"), [30_000, 2_001],
               hawk.variant(agg_strategy=1, ht=0, hash=1, wg_size=256), "xj")
    check_pair(ctx, lambda n: dg.cross_join(n=n, m=48, sink="project"), [30_000, 2_001],
               hawk.variant(proj_strategy=1, mem=1, thread_mult=64), "xp")
