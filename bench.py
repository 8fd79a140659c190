#!/usr/bin/env python3
"""Benchmark of the pipeline hot path on one MI355X.

Default run (N=1): every workload configuration, with inputs resident in HBM
before any timed region.

* The timed step (`value`, `ms_per_step`) is one pass of the wide
  scan-aggregate over 600M rows (the largest configuration): LOOP, six column
  loads, four ARITHMETIC steps, HASH_AGGREGATE of 8 aggregates into 6 groups
  with an exact 128-bit sum, result extraction, in the variant the exhaustive
  search picked. `value` is input rows per second.
* `roofline`: that step's dominant kernel, algorithmic bytes per launch over
  its average launch duration (HIP events the library records on its own
  stream during the timed steps).
* `per_pipeline`: every configuration's pipeline (selection+projection at 1M
  and 256M rows, grouped aggregation over 64M rows with 16 uniform and 1M zipf
  groups, the 120M-row star join, the wide aggregation) with rows/s,
  algorithmic GB/s, roofline fraction of the whole pipeline and of its
  dominant kernel, per-kernel times and measured HBM traffic.
* `c5`: 256 mixed pipelines as one batched graph launch, and the learned
  per-query variant picks against each query's exhaustive best and against
  Algorithm 1's per-workload variant, on queries of 4M-64M rows.
* `cpu_baseline`: the CPU oracle on all host cores and on one core, on a
  bounded sample of the timed workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "input rows/s + HBM GB/s per pipeline; learned-pick vs best-variant runtime ratio"

# variants used by the timed steps, per workload pipeline: the exhaustive
# search's best on MI355X (python bench.py --workload W --explore exhaustive),
# with its workgroup count and size re-swept for the run-time compiled kernels
DEFAULT_VARIANTS = {
    "c1": dict(proj_strategy=1, mem=1, pred=0, ht=0, hash=0, agg_strategy=0, thread_mult=1024, wg_size=256),
    "c2u": dict(proj_strategy=1, mem=1, pred=1, ht=0, hash=1, agg_strategy=0, thread_mult=1, wg_size=1024),
    "c2z": dict(proj_strategy=1, mem=1, pred=0, ht=0, hash=1, agg_strategy=0, thread_mult=1, wg_size=1024),
    "c3": dict(proj_strategy=1, mem=1, pred=0, ht=0, hash=1, agg_strategy=0, thread_mult=1, wg_size=1024),
    "c4": dict(proj_strategy=1, mem=1, pred=1, ht=0, hash=1, agg_strategy=0, thread_mult=4, wg_size=256),
}
# the 256M-row point: the best multi-pass variant of the extended space
# (the SIMD filter; the best of the paper's 32 is the same without it)
DEFAULT_VARIANTS["c1_256m"] = dict(proj_strategy=1, mem=1, pred=0, ht=0, hash=0, agg_strategy=0, thread_mult=65536,
                                   wg_size=256, filter_mode=1)

# algorithmic bytes per input row: the columns a pipeline must read once, plus
# (projection) the qualifying rows' other columns and outputs at the
# recipe's selectivity: 8 B (a, b) + 0.05 x (8 B c, d + 8 B out) = 8.8 B
ALGO_BYTES_PER_ROW = {"c1": 8.8, "c1_256m": 8.8, "c2u": 12, "c2z": 12, "c3": 24, "c4": 22}
KERNEL_FAMILIES = ["k_agg", "k_scalar_agg", "k_mp_filter", "k_mp_project", "k_sp", "k_build", "k_finalize",
                   "k_init_aggtable", "k_scan", "k_sp_concat", "k_spill_scatter", "k_spill_agg"]
WORKLOADS = {
    "all": ["c4", "c1", "c1_256m", "c2u", "c2z", "c3"],
    "c1": ["c1"],
    "c2": ["c2u", "c2z"],
    "c2u": ["c2u"],
    "c2z": ["c2z"],
    "c1_256m": ["c1_256m"],
    "c3": ["c3"],
    "c4": ["c4"],
    "c5": [],
}
DESCRIPTION = {
    "c1": "selection+projection: 1M rows, 4 int32 cols uniform [0,1000), a<100 AND 200<=b<700, out int64 c*d+a in row order",
    "c1_256m": "selection+projection scaled to 256M rows (same recipe)",
    "c2u": "grouped aggregation: 64M rows, int32 key over 16 uniform groups, int64 value [0,1e6); COUNT/SUM/MIN/MAX",
    "c2z": "grouped aggregation: 64M rows, int32 key zipf(1.1) over 1M ranks, int64 value [0,1e6); COUNT/SUM/MIN/MAX",
    "c3": "star join: 120M-row fact, 4 int32 FKs into dims 2.5k/200k/30k/80k filtered 20/5/20/1 %, SUM(int64 rev) by (d0.g, d2.g)",
    "c4": "wide scan-aggregate: 600M rows, 6 skewed groups (flag1 x flag2), 8 aggregates incl. exact 128-bit SUM(price*(100-disc)*(100+tax))",
    "c5": "mixed workload: 256 projection / aggregation / star-join pipelines over windows of 200M-row pools, "
          "lognormal rows in [1M, 200M], one batched graph launch",
}
# the timed step of each workload choice
HEADLINE = {"all": "c4", "c1": "c1", "c3": "c3", "c4": "c4", "c2u": "c2u", "c2z": "c2z", "c1_256m": "c1_256m"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_pipeline(name, rows=None):
    from paper_1709_00700_amd import datagen as dg
    if name == "c1_256m":
        tables, spec = dg.workload("c1", n=rows or (256 << 20))
    else:
        kw = {} if rows is None else {"n": rows}
        tables, spec = dg.workload(name, **kw)
    # one table namespace per pipeline
    ren = {t: f"{name}_{t}" for t in tables}
    tables = {ren[t]: c for t, c in tables.items()}
    spec["main"]["table"] = ren[spec["main"]["table"]]
    for b in spec["builds"]:
        b["table"] = ren[b["table"]]
    return tables, spec


# HBM traffic of each pipeline, from two rocprofv3 --pmc runs (FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch) of `bench.py --workload W`, summed over the
# pipeline's kernels and scaled by the ratio of known bytes to the counters'
# reading for a plain device copy (--copy-calibration: FETCH x 2.000, WRITE x
# 1.000). Valid only for the kernel sources it was measured on, with the same
# variant: reported as null otherwise.
TRAFFIC = {
    "c4": {"sources_sha": "b78525f97deeea9c", "variant_sha": "e6de8da543c2592a", "total": 13292939821,
            "per_kernel": {"k_agg": 13292905295, "k_finalize": 14335, "k_init_aggtable": 20191}},
    "c2u": {"sources_sha": "b78525f97deeea9c", "variant_sha": "c903adb01ef30859", "total": 806226194,
            "per_kernel": {"k_agg": 806202034, "k_finalize": 11808, "k_init_aggtable": 12352}},
    "c2z": {"sources_sha": "b78525f97deeea9c", "variant_sha": "366d68d5fd79efd4", "total": 1974709602,
            "per_kernel": {"k_agg": 1076107356, "k_spill_agg": 334582720, "k_spill_scatter": 562887701, "k_scan": 1118945, "k_finalize": 7944, "k_init_aggtable": 4936}},
    "c3": {"sources_sha": "b78525f97deeea9c", "variant_sha": "366d68d5fd79efd4", "total": 3434010192,
            "per_kernel": {"k_agg": 3425588047, "k_build": 6550022, "k_spill_agg": 935313, "k_scan": 139686, "k_spill_scatter": 784156, "k_finalize": 7936, "k_init_aggtable": 5032}},
    "c1_256m": {"sources_sha": "b78525f97deeea9c", "variant_sha": "e551c2cb51e36aaa", "total": 5246297115,
            "per_kernel": {"k_mp_project": 3012298547, "k_mp_filter": 2198474609, "k_scan": 35523959}},
    "c1": {"sources_sha": "b78525f97deeea9c", "variant_sha": "928f3ef35614eef6", "total": 19643731,
            "per_kernel": {"k_scan": 133597, "k_mp_filter": 8304984, "k_mp_project": 11205150}},
}
TRAFFIC_SOURCES = ["hk_agg.hip", "hk_agg_body.h", "hawk_jit.cpp", "hawk_device.h", "hawk_plan.h", "hk_proj.hip",
                   "hk_proj_body.h", "hk_common.hip", "hk_scalar.hip"]


def kernel_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1709_00700_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def variant_sha(name):
    import hashlib
    return hashlib.sha256(json.dumps(DEFAULT_VARIANTS[name], sort_keys=True).encode()).hexdigest()[:16]


def traffic_for(name):
    """Measured HBM bytes of one pass of the pipeline, per kernel, while its
    kernel sources and variant are unchanged; None otherwise."""
    t = TRAFFIC.get(name)
    if not t or t["sources_sha"] != kernel_sources_sha() or t["variant_sha"] != variant_sha(name):
        return None
    return t


def copy_calibration(nbytes):
    """A plain device copy of known size, for scaling the HBM byte counters;
    also the bandwidth that the copy and a plain read (torch's int64 sum)
    reach on this device, as practical reference points beside the peak."""
    import torch
    n = nbytes // 8
    src = torch.arange(n, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()

    def timed(f, reps=10):
        f()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            f()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    copy_ms = timed(lambda: dst.copy_(src))
    sum_ms = timed(lambda: src.sum())
    print(json.dumps({"copy_calibration_bytes": n * 8, "copies": 4,
                      "copy_gb_per_s": 2 * n * 8 / (copy_ms / 1e3) / 1e9,
                      "read_sum_gb_per_s": n * 8 / (sum_ms / 1e3) / 1e9}), flush=True)


def explore(ctx, pipes, mode, timing_db, args_limit_ms):
    from paper_1709_00700_amd import hawk
    m = hawk.HAWK_EXPLORE_EXHAUSTIVE if mode == "exhaustive" else hawk.HAWK_EXPLORE_FEATURE_WISE
    for name, q, v, nrows in pipes:
        log(f"[bench] exploring {name} ({mode})")
        best, rep = hawk.explore(ctx, [q], m, reps=2, max_iters=5, limit_ms=args_limit_ms, timing_db=timing_db,
                                 resume=bool(timing_db))
        print(json.dumps({"explore": name, "mode": mode, "rows": nrows, "best": hawk.format_variant(best),
                          "best_variant": best.as_dict(), **rep}), flush=True)


# ------------------------------------------------------------------ per-pipeline measurement
def pipeline_entry(ctx, name, q, v, nrows, reps):
    """Median pipeline time (HIP events around the whole execution) and the
    per-kernel launch durations the library records, over `reps` runs."""
    from paper_1709_00700_amd import hawk
    ms = hawk.time_variant(ctx, q, v, reps=reps)
    hawk.profile_enable(ctx, True)
    for _ in range(reps):
        hawk.execute(ctx, q, v, sync=False).free()
    stats = {f: hawk.profile_read(ctx, f) for f in KERNEL_FAMILIES}
    hawk.profile_enable(ctx, False)
    stats = {f: (t / n, n / reps) for f, (t, n) in stats.items() if n}
    dom = max(stats, key=lambda f: stats[f][0] * stats[f][1])
    algo = nrows * ALGO_BYTES_PER_ROW[name]
    entry = {"pipeline": name, "rows": nrows, "ms": ms, "rows_per_s": nrows / (ms / 1e3),
             "variant": hawk.format_variant(v), "algo_bytes": algo,
             "algo_gb_per_s": algo / (ms / 1e3) / 1e9, "frac": algo / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
             "dominant_kernel": dom, "kernel_ms": stats[dom][0],
             "kernel_frac": algo / (stats[dom][0] / 1e3) / 1e9 / HBM_PEAK_GBS,
             "kernels_ms": {f: round(s[0], 4) for f, s in stats.items()},
             "launches_per_run": {f: s[1] for f, s in stats.items()}}
    t = traffic_for(name)
    entry["traffic"] = None if t is None else {"bytes": t["total"], "per_kernel": t["per_kernel"],
                                               "vs_algo": t["total"] / algo}
    return entry


# ------------------------------------------------------------------ C5: batch and pick quality
def c5_algo_bytes(q):
    """Bytes a C5 pipeline must read (and write) at its target selectivity s:
    projection a (4 B) for every row, b, c, d (12 B) and the output (8 B) per
    qualifying row; aggregation the filter column (4 B) for every row, key and
    value (12 B) per qualifying row; star join the first key (4 B) for every
    row, each further key for the rows the probes before it keep (per-dimension
    selectivity s^(1/4)), and the revenue (8 B) per joined row."""
    n, s = q["rows"], q["selectivity"]
    if q["kind"] == 1:
        return n * (4 + s * 20)
    if q["kind"] == 2:
        return n * (4 + s * 12)
    d = s ** 0.25
    return n * (4 * (1 + d + d * d + d * d * d) + 8 * s)


def c5_batch(ctx, dev, pools_np, nq, pool_rows, schedule, autotune, steps, warmup, picker=None):
    """The 256-pipeline mixed workload as one graph replay in the tile kernels,
    also by pipeline kind; and (with a picker) with each query in its learned
    variant inside the same kind of graph."""
    import torch
    from paper_1709_00700_amd import datagen as dg
    from paper_1709_00700_amd import hawk, optimizer
    qs = dg.c5_queries(nq, pool_rows, min_rows=min(1_000_000, pool_rows), max_rows=pool_rows)
    hs = optimizer.register_c5(ctx, pools_np, qs, prefix="c5_", dev=dev)
    total_rows = sum(q["rows"] for q in qs)
    b = hawk.Batch(ctx, hs, **schedule)
    if autotune:
        best, ms = b.autotune(reps=2)
        log(f"[bench] c5: autotuned schedule {best} ({ms:.3f} ms)")
    b.run()
    r = b.result(0)
    r.info()  # raises if any hash table of the batch overflowed
    r.free()
    ms = b.time(reps=max(steps, 3))
    out = {"pipelines": nq, "rows": total_rows, "ms": ms, "rows_per_s": total_rows / (ms / 1e3),
           "schedule": b.opts(), "kinds": {}}
    b.free()
    out["algo_bytes"] = sum(c5_algo_bytes(q) for q in qs)
    out["algo_gb_per_s"] = out["algo_bytes"] / (ms / 1e3) / 1e9
    for kind in (1, 2, 3):
        sub = [h for h, q in zip(hs, qs) if q["kind"] == kind]
        rows = sum(q["rows"] for q in qs if q["kind"] == kind)
        algo = sum(c5_algo_bytes(q) for q in qs if q["kind"] == kind)
        bk = hawk.Batch(ctx, sub, **out["schedule"])
        kms = bk.time(reps=3)
        bk.free()
        out["kinds"][str(kind)] = {"pipelines": len(sub), "rows": rows, "ms": kms, "rows_per_s": rows / (kms / 1e3),
                                   "algo_bytes": algo, "algo_gb_per_s": algo / (kms / 1e3) / 1e9}
    if picker is not None:
        # every query in the variant the learned optimizer picks for it, each
        # with its own kernels as nodes of one graph (the kernels compiled
        # ahead of time, which the cost model was trained on)
        jit = getattr(ctx, "jit", False)
        ctx.set_jit(False)
        picks, _ = picker.pick(hs)
        bp = hawk.Batch(ctx, hs, variants=picks, **out["schedule"])
        pms = bp.time(reps=3)
        bp.free()
        kinds = {}
        for kind in (1, 2, 3):
            sub = [(h, v) for h, v, q in zip(hs, picks, qs) if q["kind"] == kind]
            rows = sum(q["rows"] for q in qs if q["kind"] == kind)
            bk = hawk.Batch(ctx, [h for h, _ in sub], variants=[v for _, v in sub], **out["schedule"])
            kms = bk.time(reps=3)
            bk.free()
            kinds[str(kind)] = {"ms": kms, "rows_per_s": rows / (kms / 1e3)}
        ctx.set_jit(jit)
        out["learned_variants"] = {"ms": pms, "rows_per_s": total_rows / (pms / 1e3),
                                   "algo_gb_per_s": out["algo_bytes"] / (pms / 1e3) / 1e9, "kinds": kinds,
                                   "distinct_variants": len({hawk.format_variant(v) for v in picks})}
        if jit:
            # the same picks with the run-time compiled kernels (compiled
            # before the capture, outside the timing)
            try:
                bp = hawk.Batch(ctx, hs, variants=picks, **out["schedule"])
                rms = bp.time(reps=3)
                bp.free()
                rk = {}
                for kind in (1, 2, 3):
                    sub = [(h, v) for h, v, q in zip(hs, picks, qs) if q["kind"] == kind]
                    rows = sum(q["rows"] for q in qs if q["kind"] == kind)
                    bk = hawk.Batch(ctx, [h for h, _ in sub], variants=[v for _, v in sub], **out["schedule"])
                    kms = bk.time(reps=3)
                    bk.free()
                    rk[str(kind)] = {"ms": kms, "rows_per_s": rows / (kms / 1e3)}
                out["learned_variants"]["run_time_kernels"] = {
                    "ms": rms, "rows_per_s": total_rows / (rms / 1e3),
                    "algo_gb_per_s": out["algo_bytes"] / (rms / 1e3) / 1e9, "kinds": rk}
            except hawk.HawkError as e:
                out["learned_variants"]["run_time_kernels"] = {"error": str(e)}
    torch.cuda.synchronize()
    return out


def c5_train(ctx, dev, pools_np, pool_rows, args):
    """The cost model's training timings (sampled variants of other seeded C5
    queries of 1M-64M rows over the same pools, then two rounds of active
    sampling) and the five-member ensemble trained on them."""
    from paper_1709_00700_amd import datagen as dg
    from paper_1709_00700_amd import optimizer
    hi = min(args.pq_max_rows, pool_rows)
    tr = dg.c5_queries(args.pq_train, pool_rows, dg.MASTER_SEED + 1005, min_rows=min(args.pq_min_rows // 4, hi),
                       max_rows=hi)
    tr_h = optimizer.register_c5(ctx, pools_np, tr, prefix="pqtr_", dev=dev)
    t0 = time.perf_counter()
    X, y = optimizer.training_set(ctx, tr_h, args.pq_per_query, reps=2, limit_ms=args.pq_limit_ms, seed=7,
                                  progress=lambda m: log("[bench] " + m), factor=10.0)
    t_collect = time.perf_counter() - t0
    ens = optimizer.Ensemble(ctx, size=5, penalty=1.0, seed=1)
    t0 = time.perf_counter()
    loss = ens.train(X, y, epochs=300, batch=512, lr=3e-3, seed=2)
    X, y = optimizer.refine(ctx, tr_h, ens, X, y, top=4, rounds=2, reps=2, limit_ms=args.pq_limit_ms, factor=10.0,
                            progress=lambda m: log("[bench] " + m), epochs=300, batch=512, lr=3e-3, seed=2)
    stats = {"training_samples": int(len(y)), "train_mse": loss,
             "active_sampling": "2 rounds x top 4 per training query", "collect_s": t_collect,
             "train_s": time.perf_counter() - t0}
    return ens, stats


def c5_test_queries(ctx, dev, pools_np, pool_rows, args):
    """The pick-quality queries (4M-64M rows), kinds in turn, so that a search
    cut short by the time budget still covers each kind."""
    from paper_1709_00700_amd import datagen as dg
    from paper_1709_00700_amd import optimizer
    hi = min(args.pq_max_rows, pool_rows)
    te = dg.c5_queries(args.pq_test, pool_rows, dg.MASTER_SEED + 5 + 77, min_rows=min(args.pq_min_rows, hi),
                       max_rows=hi)
    by_kind = [[q for q in te if q["kind"] == k] for k in (1, 2, 3)]
    te = [q for grp in zip(*[g + [None] * (len(te) - len(g)) for g in by_kind]) for q in grp if q is not None]
    return te, optimizer.register_c5(ctx, pools_np, te, prefix="pqte_", dev=dev)


def c5_pick_quality(ctx, te, te_h, ens, alg1, picker, train_stats, t_alg1, args, t_start):
    """The learned per-query picks on C5 queries of 4M-64M rows (their best
    variants are HBM-bound), against each query's exhaustive best (pruned at
    10x the running best) and Algorithm 1's per-kind variant; then the same
    queries back to back in their best variants against one batch replay in
    the tile kernels, in the picked variants and in the best variants."""
    from paper_1709_00700_amd import hawk, optimizer
    t0 = time.perf_counter()
    deadline = t_start + args.pq_budget_s
    # one timed run per variant in the search; the search's best and the picks
    # are then timed again with 5 runs each and compared on those times
    pq = optimizer.pick_quality(ctx, te_h, picker, reps=1, limit_ms=args.pq_limit_ms, alg1=alg1,
                                progress=lambda m: log("[bench] " + m),
                                extra={"ensemble": ens, "single_model": ens.models[0]},
                                factor=10.0, deadline=deadline, confirm_reps=5)
    t_ex = time.perf_counter() - t0
    done = pq["queries"]
    rows = pq.pop("per_query")
    for q, r in zip(te[:done], rows):
        r.update({"kind": q["kind"], "rows": q["rows"]})
    # the same queries back to back in their exhaustive-best variants (each a
    # separate execution: host launches included), against batch replays
    best_vs = []
    for h, r in zip(te_h[:done], rows):
        best_vs.append(next(v for v in hawk.variant_space(h) if optimizer.variant_key(h, v) == r["best"]))
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for h, v in zip(te_h[:done], best_vs):
        hawk.execute(ctx, h, v).free()
    seq = []
    for _ in range(3):
        e0.record(ctx.stream)
        res = [hawk.execute(ctx, h, v, sync=False) for h, v in zip(te_h[:done], best_vs)]
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        for r_ in res:
            r_.free()
        seq.append(e0.elapsed_time(e1))
    sched = dict(tile_rows_log2=17, wgs_per_cu=8, order=0)
    batch = {}
    for name, vs in (("tile", None), ("picked", picker.pick(te_h[:done])[0]), ("best", best_vs)):
        b = hawk.Batch(ctx, te_h[:done], variants=vs, **sched)
        batch[name] = b.time(reps=3)
        b.free()
    pq.update(train_stats)
    pq.update({"alg1_s": t_alg1, "exhaustive_s": t_ex, "pool_rows": args.rows or args.c5_pool_rows,
               "rows_range": [min(q["rows"] for q in te), max(q["rows"] for q in te)],
               "best_ms_median": float(sorted(r["best_ms"] for r in rows)[len(rows) // 2]) if rows else None,
               "prune": "a variant slower than 10x the fastest measured so far for the query is +inf",
               "confirm": "the search's best and every pick timed again (5 runs each) and compared on those times",
               "alg1_variants": {str(k): hawk.format_variant(v) for k, (v, _) in alg1.items()},
               "picker": "ensemble of 5 cost models (mean + 1 sd of predicted ln(ms)) proposes one variant per "
                         "query; a race of 2 timed runs each against Algorithm 1's variant for the query's kind "
                         "keeps the faster",
               "race_ms": picker.race_ms,
               "kernels": "compiled ahead of time (run-time compilation off for the whole evaluation)",
               "sum_best_ms": sum(r["best_ms"] for r in rows),
               "sum_best_sequential_ms": sorted(seq)[1],
               "batch_ms": batch["tile"], "batch_picked_ms": batch["picked"], "batch_best_ms": batch["best"],
               "per_query": rows})
    return pq


# ------------------------------------------------------------------ CPU baseline
def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def same_answer(got, ref):
    """The device's answer equals the oracle's (AVG within 1e-12 relative)."""
    import numpy as np
    if got["rows"] != ref["rows"]:
        return False
    if "cols" in ref:
        return all(np.array_equal(np.asarray(a), np.asarray(b)) for a, b in zip(got["cols"], ref["cols"]))
    if not all(np.array_equal(np.asarray(a), np.asarray(b)) for a, b in zip(got["keys"], ref["keys"])):
        return False
    if not np.array_equal(np.asarray(got["count"]), np.asarray(ref["count"])):
        return False
    for a, b in zip(got["aggs"], ref["aggs"]):
        for u, v in zip(list(a), list(b)):
            if isinstance(u, float) or isinstance(v, float):
                if not ((u != u and v != v) or abs(u - v) <= 1e-12 * abs(v)):
                    return False
            elif int(u) != int(v):
                return False
    return True


def cpu_baseline(name, budget_s=15.0, ctx=None, variant=None):
    """The oracle as it stands on a bounded sample of the timed workload (its
    first n rows, n doubling from 2^20 while the budget lasts): on all host
    cores of this GPU's share (row-partitioned: contiguous ranges, one thread
    each, partial results merged), and on one core. With ctx, the largest
    sample also runs on the device in the timed variant and its answer is
    compared element by element with the oracle's."""
    import oracle
    from paper_1709_00700_amd import datagen as dg
    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:
        share = os.cpu_count() or 1
    threads = max(1, min(share, 16))
    out = {}
    for leg, th in (("all", threads), ("one", 1)):
        rows_done, secs, samples, last = 0, 0.0, [], 0.0
        n = 1 << 20
        # the next sample (twice the rows) is taken while it should end within the budget
        keep = None
        while (not samples or secs + 2.2 * last <= budget_s) and n <= (1 << 28):
            tables, spec = make_pipeline(name, rows=n)
            t0 = time.perf_counter()
            ref = oracle.run(tables, spec, threads=th)
            last = time.perf_counter() - t0
            secs += last
            rows_done += n
            samples.append(n)
            keep = (tables, spec, ref, n) if leg == "all" else None
            del tables
            n *= 2
        if keep is not None and ctx is not None:
            from paper_1709_00700_amd import hawk
            tables, spec, ref, nv = keep
            ren = {t: "verify_" + t for t in tables}
            spec["main"]["table"] = ren[spec["main"]["table"]]
            for b in spec["builds"]:
                b["table"] = ren[b["table"]]
            ctx.register_numpy({ren[t]: c for t, c in tables.items()})
            r = hawk.execute(ctx, hawk.build_query(ctx, spec), variant)
            got = r.to_numpy(spec)
            r.free()
            out["verify"] = {"rows": nv, "matches_oracle": same_answer(got, ref)}
        keep = None
        out[leg] = {"value": rows_done / secs, "cores": th, "seconds": secs,
                    "sample": f"first rows of the same seeded {name} workload, n = {samples[0]}..{samples[-1]} "
                              f"doubling ({rows_done} rows in all)"}
    res = {"value": out["all"]["value"], "unit": "rows/s", "cores": out["all"]["cores"], "kind": "oracle",
           "sample": out["all"]["sample"] + ", row-partitioned over threads",
           "single_core": {"value": out["one"]["value"], "cores": 1, "sample": out["one"]["sample"]},
           "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity": share}}
    if "verify" in out:
        res["verified"] = out["verify"]
    return res


# ------------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="all", choices=sorted(WORKLOADS))
    ap.add_argument("--rows", type=int, default=None, help="override the input rows per pipeline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds per CPU baseline leg")
    ap.add_argument("--no-c5", action="store_true", help="all: skip the mixed workload")
    ap.add_argument("--no-pick-quality", action="store_true", help="skip the learned-pick evaluation")
    ap.add_argument("--explore", choices=["exhaustive", "feature_wise"], default=None,
                    help="run the variant optimizer on each pipeline instead of the timed steps")
    ap.add_argument("--timing-db", default=None, help="append every exploration measurement to this file (and resume)")
    ap.add_argument("--explore-limit-ms", type=float, default=200.0, help="pruning limit of the exploration")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (HBM counter calibration)")
    ap.add_argument("--no-jit", action="store_true", help="use only the kernels compiled ahead of time")
    ap.add_argument("--c5-queries", type=int, default=256)
    ap.add_argument("--c5-pool-rows", type=int, default=200_000_000)
    ap.add_argument("--autotune", action="store_true", help="c5: autotune the batch schedule first")
    ap.add_argument("--pq-train", type=int, default=32)
    ap.add_argument("--pq-test", type=int, default=16)
    ap.add_argument("--pq-per-query", type=int, default=40)
    ap.add_argument("--pq-min-rows", type=int, default=4_000_000)
    ap.add_argument("--pq-max-rows", type=int, default=64_000_000)
    ap.add_argument("--pq-limit-ms", type=float, default=100.0)
    ap.add_argument("--pq-budget-s", type=float, default=330.0, help="wall budget of the pick-quality leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs each pipeline on one GPU "
              "(across several, a pipeline would shard by row ranges of its scanned table)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1709_00700_amd import hawk

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    t_run = time.perf_counter()
    ctx = hawk.Context(0)
    if not args.no_jit and not args.explore:
        ctx.set_jit(True)  # aggregation kernels compiled for each plan structure during the warm-up
    ncu, lds_bytes = ctx.device_info()
    log(f"[bench] device: {ncu} compute units, {lds_bytes} LDS bytes per workgroup")
    out = {}
    pipes = []
    for name in WORKLOADS[args.workload]:
        log(f"[bench] generating + uploading {name}")
        tables, spec = make_pipeline(name, args.rows)
        ctx.register_numpy(tables)
        q = hawk.build_query(ctx, spec)
        v = hawk.variant(**DEFAULT_VARIANTS[name])
        nrows = len(next(iter(tables[spec["main"]["table"]].values())))
        pipes.append((name, q, v, nrows))
        del tables
    if args.explore:
        explore(ctx, pipes, args.explore, args.timing_db, args.explore_limit_ms)
        ctx.close()
        return
    # every pipeline once, checked end to end (and its run-time kernel compiled)
    for name, q, v, _ in pipes:
        r = hawk.execute(ctx, q, v)
        r.info()
        r.free()

    head = HEADLINE.get(args.workload)
    if head is None:
        head_pipes = pipes
        workload_desc = DESCRIPTION["c2u"] + "; and " + DESCRIPTION["c2z"] if args.workload == "c2" else None
    else:
        head_pipes = [p for p in pipes if p[0] == head]
        workload_desc = DESCRIPTION[head]
    stream = ctx.stream
    per, value, ms_per_step, roofline, wall = [], None, None, None, None
    if head_pipes:
        def step():
            for _, q, v, _ in head_pipes:
                hawk.execute(ctx, q, v, sync=False).free()

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        log(f"[bench] timing {args.steps} steps of {[p[0] for p in head_pipes]}")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        # the library brackets each of its launches with HIP events on its own
        # stream while the timed steps run: the roofline's kernel durations
        hawk.profile_enable(ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms_per_step = e0.elapsed_time(e1) / args.steps
        step_rows = sum(p[3] for p in head_pipes)
        value = step_rows / (ms_per_step / 1e3)
        timed = {f: hawk.profile_read(ctx, f) for f in KERNEL_FAMILIES}
        hawk.profile_enable(ctx, False)
        # dominant kernel of the timed steps: algorithmic bytes per launch
        # (one launch per pipeline per step) over its average launch duration
        dom = max(timed, key=lambda f: timed[f][0])
        tot_ms, nl = timed[dom]
        avg_ms = tot_ms / nl
        algo = sum(p[3] * ALGO_BYTES_PER_ROW[p[0]] for p in head_pipes) / len(head_pipes)
        achieved = algo / (avg_ms / 1e3) / 1e9
        tr = [traffic_for(p[0]) for p in head_pipes]
        traffic = None
        if all(t is not None for t in tr):
            traffic = sum(t["per_kernel"].get(dom, 0) for t in tr) / len(tr)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "algo_bytes_per_launch": algo, "avg_launch_ms": round(avg_ms, 4), "launches_timed": nl}
    for name, q, v, nrows in pipes:
        log(f"[bench] pipeline {name}")
        per.append(pipeline_entry(ctx, name, q, v, nrows, reps=max(5, args.steps // 2)))
    if args.workload in ("all", "c5") and not args.no_c5:
        from paper_1709_00700_amd import datagen as dg
        from paper_1709_00700_amd import optimizer
        pool_rows = args.rows or args.c5_pool_rows
        log(f"[bench] c5: generating + uploading pools of {pool_rows} rows")
        pools_np = dg.c5_pools(pool_rows)
        dev = optimizer.upload_pools(ctx, pools_np)
        picker, ens = None, None
        if not args.no_pick_quality:
            t_start = time.perf_counter()
            ctx.set_jit(False)  # the optimizer times the kernels compiled ahead of time
            log("[bench] c5: cost model training")
            ens, train_stats = c5_train(ctx, dev, pools_np, pool_rows, args)
            te, te_h = c5_test_queries(ctx, dev, pools_np, pool_rows, args)
            t0 = time.perf_counter()
            alg1 = optimizer.alg1_per_kind(ctx, te_h, reps=2, limit_ms=args.pq_limit_ms)
            t_alg1 = time.perf_counter() - t0
            # the per-query optimizer: the ensemble's pick, raced on the query
            # against Algorithm 1's variant for the query's kind
            picker = optimizer.WithFallback(ens, {k: v for k, (v, _) in alg1.items()}, race_ctx=ctx)
            ctx.set_jit(not args.no_jit)
        log("[bench] c5: batch")
        sched = dict(tile_rows_log2=17, wgs_per_cu=8, order=0)
        c5 = c5_batch(ctx, dev, pools_np, args.c5_queries, pool_rows, sched, args.autotune, args.steps,
                      args.warmup, picker=picker)
        c5["codegen"] = dict(zip(("run_time_kernels", "compile_ms"), ctx.jit_stats()))
        if picker is not None:
            log("[bench] c5: pick quality")
            ctx.set_jit(False)
            c5["pick_quality"] = c5_pick_quality(ctx, te, te_h, ens, alg1, picker, train_stats, t_alg1, args,
                                                 t_start)
            ctx.set_jit(not args.no_jit)
            ens.free()
        out["c5"] = c5
        del pools_np
        if not head_pipes:
            value, ms_per_step, workload_desc = c5["rows_per_s"], c5["ms"], DESCRIPTION["c5"]
    res = {"metric": METRIC, "value": value, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": workload_desc, "timed_pipelines": [p[0] for p in head_pipes],
                      "rows_per_step": sum(p[3] for p in head_pipes), "compute_units": ncu,
                      "codegen": dict(zip(("run_time_kernels", "compile_ms"), ctx.jit_stats()),
                                      run_time=not args.no_jit)},
           "roofline": roofline, "per_pipeline": per, **out, "wall_s_timed": wall}
    if not args.no_cpu_baseline and head_pipes:
        log("[bench] cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(head_pipes[0][0], args.cpu_budget, ctx, head_pipes[0][2])
    res["run_s"] = time.perf_counter() - t_run
    print(json.dumps(res), flush=True)
    ctx.close()
    if not res.get("cpu_baseline", {}).get("verified", {}).get("matches_oracle", True):
        print("bench.py: the device's answer on the baseline sample differs from the oracle's", file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
