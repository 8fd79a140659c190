#!/usr/bin/env python3
"""Benchmark of the pipeline hot path on one MI355X.

A step is one pass of the whole hot path over the configured workload: every
pipeline of the workload runs once (build pipelines, scan, selection, probes,
arithmetic, aggregation or projection, result extraction) in the variant the
variant optimizer picked for it. Inputs are resident in HBM before the timed
region; K steps are timed between stream synchronisations.

Default workload (N=1): grouped aggregation over 64M rows with an int32 key
and an int64 value, COUNT/SUM/MIN/MAX per group, once with 16 uniform groups
and once with zipf(1.1) keys over 1M ranks (the two grouped-aggregation
cases). `value` is input rows per second of the whole step.

Also reported: the dominant kernel's roofline (algorithmic bytes per launch /
its average launch duration, timed live with HIP events on the library's
stream), per-pipeline rows/s and GB/s, and the CPU oracle timed on a bounded
sample of the same workload on the host.
"""
from __future__ import annotations

import argparse
import json
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
    "c3": dict(proj_strategy=1, mem=1, pred=0, ht=0, hash=1, agg_strategy=0, thread_mult=8, wg_size=512),
    "c4": dict(proj_strategy=1, mem=1, pred=1, ht=0, hash=1, agg_strategy=0, thread_mult=8, wg_size=512),
}

# algorithmic bytes read per input row of each pipeline (columns the
# pipeline must read once), plus the kernel family that dominates it
ALGO_BYTES_PER_ROW = {"c1": None, "c2u": 12, "c2z": 12, "c3": 24, "c4": 22}
KERNEL_FAMILIES = ["k_agg", "k_scalar_agg", "k_mp_filter", "k_mp_project", "k_sp", "k_build", "k_finalize",
                   "k_init_aggtable", "k_scan", "k_sp_concat", "k_spill_scatter", "k_spill_agg"]
WORKLOADS = {
    "c1": ["c1"],
    "c2": ["c2u", "c2z"],
    "c3": ["c3"],
    "c4": ["c4"],
    "c5": [],
}
DESCRIPTION = {
    "c1": "selection+projection: 1M rows, 4 int32 cols uniform [0,1000), a<100 AND 200<=b<700, out int64 c*d+a in row order",
    "c2": "grouped aggregation: 64M rows int32 key + int64 value uniform [0,1e6); 16 uniform groups and zipf(1.1) over 1M ranks; COUNT/SUM/MIN/MAX",
    "c3": "star join: 120M-row fact, 4 int32 FKs into dims 2.5k/200k/30k/80k filtered 20/5/20/1 %, SUM(int64 rev) by (d0.g, d2.g)",
    "c4": "wide scan-aggregate: 600M rows, 6 skewed groups, 8 aggregates incl. exact 128-bit SUM(price*(100-disc)*(100+tax))",
    "c5": "mixed workload: 256 projection / aggregation / star-join pipelines over windows of 200M-row pools, "
          "lognormal rows in [1M, 200M], one batched graph launch",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_pipelines(workload, rows):
    from paper_1709_00700_amd import datagen as dg
    out = []
    for name in WORKLOADS[workload]:
        kw = {} if rows is None else {"n": rows}
        tables, spec = dg.workload(name, **kw)
        # one table namespace per pipeline
        ren = {t: f"{name}_{t}" for t in tables}
        tables = {ren[t]: c for t, c in tables.items()}
        spec["main"]["table"] = ren[spec["main"]["table"]]
        for b in spec["builds"]:
            b["table"] = ren[b["table"]]
        out.append((name, tables, spec))
    return out


# HBM traffic of the dominant kernel per workload, from two rocprofv3 --pmc
# runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) of that workload, each
# scaled by the ratio of known bytes to the counter's reading for a plain
# device copy (--copy-calibration). Valid only for the kernel sources it was
# measured on, with the same variants: bench.py reports null otherwise.
TRAFFIC = {
    ("k_agg", "c2"): {"sources_sha": "28f9545bf8c32692", "variants_sha": "c62b14057a3f9b21",
                      "bytes_per_launch": 981707435},
    ("k_agg", "c3"): {"sources_sha": "28f9545bf8c32692", "variants_sha": "4da2aec3e3d4646d",
                      "bytes_per_launch": 3330324547},
    ("k_agg", "c4"): {"sources_sha": "28f9545bf8c32692", "variants_sha": "eb3f0a286c66bac6",
                      "bytes_per_launch": 13333290310},
}


def kernel_sources_sha(kernel):
    import hashlib
    files = {"k_agg": ["hk_agg.hip", "hk_agg_body.h", "hawk_jit.cpp", "hawk_device.h", "hawk_plan.h"]}.get(kernel, [])
    if not files:
        return None
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1709_00700_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def variants_sha(workload):
    import hashlib
    return hashlib.sha256(json.dumps([DEFAULT_VARIANTS[p] for p in WORKLOADS[workload]],
                                     sort_keys=True).encode()).hexdigest()[:16]


def traffic_for(kernel, workload):
    """Measured HBM bytes per launch, while the kernel sources and the workload's variants are unchanged."""
    t = TRAFFIC.get((kernel, workload))
    if not t or t["sources_sha"] != kernel_sources_sha(kernel) or t.get("variants_sha") != variants_sha(workload):
        return None
    return t["bytes_per_launch"]


def copy_calibration(nbytes):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = nbytes // 8
    src = torch.arange(n, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 8, "copies": 4}), flush=True)


def explore(ctx, pipes, mode, timing_db, args_limit_ms):
    from paper_1709_00700_amd import hawk
    m = hawk.HAWK_EXPLORE_EXHAUSTIVE if mode == "exhaustive" else hawk.HAWK_EXPLORE_FEATURE_WISE
    for name, q, v, nrows in pipes:
        log(f"[bench] exploring {name} ({mode})")
        best, rep = hawk.explore(ctx, [q], m, reps=2, max_iters=5, limit_ms=args_limit_ms, timing_db=timing_db)
        print(json.dumps({"explore": name, "mode": mode, "rows": nrows, "best": hawk.format_variant(best),
                          "best_variant": best.as_dict(), **rep}), flush=True)


def run_c5(args):
    """Mixed workload: every pipeline in one batched graph launch (rows/s of the
    whole batch); with --pick-quality also the learned per-query picks against
    exhaustive search and Algorithm 1, on a smaller seeded instance."""
    import torch
    from paper_1709_00700_amd import datagen as dg
    from paper_1709_00700_amd import hawk, optimizer

    pool_rows = args.rows or 200_000_000
    nq = args.c5_queries
    ctx = hawk.Context(0)
    if not args.no_jit:
        ctx.set_jit(True)
    ncu, _ = ctx.device_info()
    log(f"[bench] c5: generating pools of {pool_rows} rows, {nq} pipelines")
    pools = dg.c5_pools(pool_rows)
    qs = dg.c5_queries(nq, pool_rows, min_rows=min(1_000_000, pool_rows), max_rows=pool_rows)
    hs = optimizer.register_c5(ctx, pools, qs)
    del pools
    total_rows = sum(q["rows"] for q in qs)
    log("[bench] c5: capturing the batch")
    b = hawk.Batch(ctx, hs)
    if args.autotune:
        best, ms = b.autotune(reps=2)
        log(f"[bench] c5: autotuned schedule {best} ({ms:.3f} ms)")
    b.run()
    r = b.result(0)
    r.info()  # raises if any hash table of the batch overflowed
    r.free()
    for _ in range(args.warmup):
        b.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(ctx.stream)
    for _ in range(args.steps):
        b.run()
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    out = {"metric": METRIC, "value": total_rows / (ms / 1e3), "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": DESCRIPTION["c5"], "pipelines": nq, "rows_per_step": total_rows,
                      "pool_rows": pool_rows, "schedule": b.opts(), "compute_units": ncu,
                      "codegen": dict(zip(("run_time_kernels", "compile_ms"), ctx.jit_stats()),
                                      run_time=not args.no_jit),
                      "kinds": {k: sum(1 for q in qs if q["kind"] == k) for k in (1, 2, 3)}},
           "wall_s_timed": wall}
    b.free()
    if args.pick_quality:
        out["pick_quality"] = c5_pick_quality(ctx, args)
    print(json.dumps(out), flush=True)
    ctx.close()


def c5_pick_quality(ctx, args):
    """Train the cost model on sampled-variant timings of one seeded C5 instance,
    then compare its per-query picks and Algorithm 1's per-kind variant with the
    exhaustive best of each query of another instance."""
    from paper_1709_00700_amd import datagen as dg
    from paper_1709_00700_amd import hawk, optimizer

    pool = args.pq_pool_rows
    lim = args.pq_limit_ms
    # the optimizer measures the kernels compiled ahead of time (compiling
    # every variant of every plan at run time would dominate the search)
    ctx.set_jit(False)
    seed_train, seed_test = dg.MASTER_SEED + 1005, dg.MASTER_SEED + 5
    log(f"[bench] pick quality: pools of {pool} rows, {args.pq_train} training / {args.pq_test} test pipelines")
    tr_pools = dg.c5_pools(pool, seed_train)
    tr = dg.c5_queries(args.pq_train, pool, seed_train, min_rows=min(10_000, pool), max_rows=pool)
    tr_h = optimizer.register_c5(ctx, tr_pools, tr, prefix="train_")
    del tr_pools
    te_pools = dg.c5_pools(pool, seed_test)
    te = dg.c5_queries(args.pq_test, pool, seed_test, min_rows=min(10_000, pool), max_rows=pool)
    te_h = optimizer.register_c5(ctx, te_pools, te, prefix="test_")
    del te_pools
    t0 = time.perf_counter()
    X, y = optimizer.training_set(ctx, tr_h, args.pq_per_query, reps=2, limit_ms=lim, seed=7,
                                  progress=lambda m: log("[bench] " + m))
    t_collect = time.perf_counter() - t0
    log(f"[bench] pick quality: {len(y)} training samples in {t_collect:.1f} s")
    # the picks come from an ensemble of five models (mean + one standard
    # deviation of their predictions); a single model is scored beside it
    ens = optimizer.Ensemble(ctx, size=5, penalty=1.0, seed=1)
    t0 = time.perf_counter()
    loss = ens.train(X, y, epochs=300, batch=512, lr=3e-3, seed=2)
    t_train = time.perf_counter() - t0
    single = ens.models[0]
    t0 = time.perf_counter()
    alg1 = optimizer.alg1_per_kind(ctx, te_h, reps=2, limit_ms=lim)
    t_alg1 = time.perf_counter() - t0
    log("[bench] pick quality: exhaustive search of the test pipelines")
    t0 = time.perf_counter()
    pq = optimizer.pick_quality(ctx, te_h, ens, reps=2, limit_ms=lim, alg1=alg1,
                                progress=lambda m: log("[bench] " + m), extra={"single_model": single})
    t_ex = time.perf_counter() - t0
    pq.update({"training_samples": int(len(y)), "train_mse": loss, "collect_s": t_collect, "train_s": t_train,
               "alg1_s": t_alg1, "exhaustive_s": t_ex, "pool_rows": pool,
               "alg1_variants": {str(k): hawk.format_variant(v) for k, (v, _) in alg1.items()},
               "alg1_evaluated": {str(k): r["evaluated"] for k, (_, r) in alg1.items()},
               "picker": "ensemble of 5 cost models, mean + 1 sd of predicted ln(ms)"})
    ens.free()
    return pq


def cpu_baseline(workload, budget_s=20.0):
    """The oracle as it stands, single-threaded, on a bounded sample of the workload."""
    import oracle
    from paper_1709_00700_amd import datagen as dg
    rows_done, secs, samples = 0, 0.0, []
    names = WORKLOADS[workload]
    n = 1 << 20
    while secs < budget_s and n <= (1 << 26):
        for name in names:
            tables, spec = dg.workload(name, n=n) if name != "c3" else dg.workload(name, n=n)
            t0 = time.perf_counter()
            oracle.run(tables, spec)
            dt = time.perf_counter() - t0
            rows_done += n
            secs += dt
            samples.append(f"{name}:{n}")
        n *= 2
    return {"value": rows_done / secs, "unit": "rows/s", "cores": 1, "kind": "oracle",
            "sample": f"first rows of the same seeded workload: {', '.join(samples)} ({secs:.1f} s total)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--rows", type=int, default=None, help="override the input rows per pipeline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--explore", choices=["exhaustive", "feature_wise"], default=None,
                    help="run the variant optimizer on each pipeline instead of the timed steps")
    ap.add_argument("--timing-db", default=None, help="append every exploration measurement to this file")
    ap.add_argument("--explore-limit-ms", type=float, default=200.0, help="pruning limit of the exploration")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (HBM counter calibration)")
    ap.add_argument("--no-jit", action="store_true", help="use only the kernels compiled ahead of time")
    ap.add_argument("--c5-queries", type=int, default=256)
    ap.add_argument("--autotune", action="store_true", help="c5: autotune the batch schedule first")
    ap.add_argument("--pick-quality", action="store_true", help="c5: also evaluate the learned per-query picks")
    ap.add_argument("--pq-pool-rows", type=int, default=2_000_000)
    ap.add_argument("--pq-train", type=int, default=48)
    ap.add_argument("--pq-test", type=int, default=24)
    ap.add_argument("--pq-per-query", type=int, default=64)
    ap.add_argument("--pq-limit-ms", type=float, default=10.0)
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
    if args.workload == "c5":
        run_c5(args)
        return
    ctx = hawk.Context(0)
    if not args.no_jit and not args.explore:
        ctx.set_jit(True)  # aggregation kernels compiled for each plan structure during the warm-up
    ncu, lds_bytes = ctx.device_info()
    log(f"[bench] device: {ncu} compute units, {lds_bytes} LDS bytes per workgroup")
    pipes = []
    total_rows = 0
    for name, tables, spec in make_pipelines(args.workload, args.rows):
        log(f"[bench] generating + uploading {name}")
        ctx.register_numpy(tables)
        q = hawk.build_query(ctx, spec)
        v = hawk.variant(**DEFAULT_VARIANTS[name])
        nrows = len(next(iter(tables[spec["main"]["table"]].values())))
        total_rows += nrows
        pipes.append((name, q, v, nrows))
        del tables
    stream = ctx.stream
    if args.explore:
        explore(ctx, pipes, args.explore, args.timing_db, args.explore_limit_ms)
        ctx.close()
        return

    def step():
        for _, q, v, _ in pipes:
            hawk.execute(ctx, q, v, sync=False).free()

    # warm-up, checked end to end once
    for name, q, v, _ in pipes:
        r = hawk.execute(ctx, q, v)
        r.info()
        r.free()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
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
    value = total_rows / (ms_per_step / 1e3)
    timed = {f: hawk.profile_read(ctx, f) for f in KERNEL_FAMILIES}
    hawk.profile_enable(ctx, False)

    # per-pipeline times and the dominant kernel, timed with events on the library stream
    per = []
    kern_stats = {}
    for name, q, v, nrows in pipes:
        ms = hawk.time_variant(ctx, q, v, reps=max(5, args.steps // 2))
        hawk.profile_enable(ctx, True)
        for _ in range(max(5, args.steps // 2)):
            hawk.execute(ctx, q, v, sync=False).free()
        stats = {f: hawk.profile_read(ctx, f) for f in KERNEL_FAMILIES}
        hawk.profile_enable(ctx, False)
        stats = {f: (t / n, n) for f, (t, n) in stats.items() if n}
        dom = max(stats, key=lambda f: stats[f][0])
        bpr = ALGO_BYTES_PER_ROW[name]
        entry = {"pipeline": name, "rows": nrows, "ms": ms, "rows_per_s": nrows / (ms / 1e3),
                 "variant": hawk.format_variant(v), "dominant_kernel": dom, "kernel_ms": stats[dom][0],
                 "kernels_ms": {f: round(s[0], 4) for f, s in stats.items()}}
        if bpr:
            entry["algo_gb_per_s"] = nrows * bpr / (ms / 1e3) / 1e9
            entry["kernel_algo_gb_per_s"] = nrows * bpr / (stats[dom][0] / 1e3) / 1e9
        per.append(entry)
        kern_stats.setdefault(dom, []).append((stats[dom][0], nrows * (bpr or 0)))
    # roofline of the dominant kernel of the timed steps: algorithmic bytes
    # per launch (the pipelines' launches are equally many) / the average
    # launch duration recorded during the timed region
    dom = max(timed, key=lambda f: timed[f][0])
    tot_ms, nl = timed[dom]
    avg_ms = tot_ms / nl
    launches = [b for _, b in kern_stats.get(dom, [])]
    avg_bytes = sum(launches) / len(launches) if launches else 0.0
    achieved = avg_bytes / (avg_ms / 1e3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_for(dom, args.workload),
                "algo_bytes_per_launch": avg_bytes, "avg_launch_ms": round(avg_ms, 4), "launches_timed": nl}

    out = {"metric": METRIC, "value": value, "unit": "rows/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": DESCRIPTION[args.workload], "pipelines": [p[0] for p in pipes],
                      "rows_per_step": total_rows, "compute_units": ncu,
                      "codegen": dict(zip(("run_time_kernels", "compile_ms"), ctx.jit_stats()),
                                      run_time=not args.no_jit)},
           "roofline": roofline, "per_pipeline": per, "wall_s_timed": wall}
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_budget)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
