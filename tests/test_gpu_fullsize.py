"""GPU parity at the workloads' full sizes, in the variants and launch
configuration the benchmark times (kernels compiled at run time for each
plan), element by element against the oracle: grouped aggregation over 64M
rows (16 uniform groups; zipf over 1M ranks), the 120M-row star join, the
wide aggregation at 600M rows and a 64M-row stress instance whose 128-bit
sums pass 2^63, and spilling at sizes where every workgroup regroups its
spilled rows in many 8192-entry tiles."""
import os

import numpy as np
import pytest

import oracle
from gpu_common import compare, say
from paper_1709_00700_amd import datagen as dg
from paper_1709_00700_amd import hawk

import bench

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hawk.Context(0)
    c.set_jit(True)
    yield c
    c.close()


def oracle_threads():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(16, os.cpu_count() or 1))


def run_one(ctx, tables, spec, v, label):
    say(label, "oracle")
    # row ranges on the host cores, merged exactly (pinned to the one-thread answer)
    ref = oracle.run(tables, spec, threads=oracle_threads())
    say(label, "device run", hawk.format_variant(v))
    dev = ctx.register_numpy(tables)
    q = hawk.build_query(ctx, spec)
    r = hawk.execute(ctx, q, v)
    got = r.to_numpy(spec)
    r.free()
    compare(got, ref, spec, label)
    del dev
    say(label, "rows", ref["rows"], "ok")
    return ref


@pytest.mark.parametrize("name", ["c2u", "c2z", "c3"])
def test_full_size_in_bench_variant(ctx, name):
    tables, spec = dg.workload(name)
    run_one(ctx, tables, spec, hawk.variant(**bench.DEFAULT_VARIANTS[name]), f"{name} full size")


def test_c4_full_size_in_bench_variant(ctx):
    tables, spec = dg.workload("c4")
    assert len(tables["t"]["qty"]) == 600_000_000
    run_one(ctx, tables, spec, hawk.variant(**bench.DEFAULT_VARIANTS["c4"]), "c4 600M")


def test_c4_64m_sums_past_int64(ctx):
    tables, spec = dg.c4_wide(n=64 << 20, price_hi=1 << 40)
    ref = run_one(ctx, tables, spec, hawk.variant(**bench.DEFAULT_VARIANTS["c4"]), "c4 64M price<2^40")
    assert max(int(x) for x in ref["aggs"][4]) > (1 << 63)


def spill_variant():
    # the zipf pipeline's variant: one workgroup of 1024 threads per CU, local
    # LDS tables with linear probing, so rows that miss the table spill
    return hawk.variant(**bench.DEFAULT_VARIANTS["c2z"])


def test_spill_distinct_keys_many_tiles_per_workgroup(ctx):
    """8M rows with pairwise distinct keys. A key's only row is the one that
    can put it into a workgroup's LDS table, so at most one row per table slot
    is aggregated in LDS: a workgroup of R rows spills at least R - LC of
    them, LC <= 4096 slots (160 KiB over 40-byte slots). With 256 workgroups
    R = 32768, so every workgroup spills at least 28672 entries, which its
    regrouping moves in at least four 8192-entry tiles."""
    ncu, _ = ctx.device_info()
    n = 8 << 20
    keys = dg.sparse_keys(dg.MASTER_SEED, 0x7001, n)
    assert len(np.unique(keys)) == n
    v = dg.uniform(dg.MASTER_SEED, 0x7002, n, -(1 << 40), 1 << 40, np.int64)
    spec = {"builds": [], "main": {"table": "t", "filters": [], "probes": [], "arith": [],
                                   "group_by": ["k"],
                                   "aggs": [("count", None, False), ("sum", "v", False),
                                            ("min", "v", False), ("max", "v", False)],
                                   "groups_hint": n}}
    var = spill_variant()
    rows_per_wg = n // (var.thread_mult * ncu)
    assert rows_per_wg - 4096 > 3 * 8192
    say("distinct keys: rows per workgroup", rows_per_wg, "spilled at least", rows_per_wg - 4096)
    run_one(ctx, {"t": {"k": keys, "v": v}}, spec, var, "spill distinct keys")
    ctx.set_jit(False)
    run_one(ctx, {"t2": {"k": keys, "v": v}}, {**spec, "main": {**spec["main"], "table": "t2"}}, var,
            "spill distinct keys, precompiled")


def test_spill_zipf_16m(ctx):
    tables, spec = dg.c2_aggregation(n=16 << 20, dist="zipf", nranks=1_000_000)
    run_one(ctx, tables, spec, spill_variant(), "c2z 16M")
