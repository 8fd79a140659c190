"""Variant selection over a workload of many pipelines (Section 8, and the
per-query optimizer the paper leaves to future work in Sections 9.3.4 and 9.4).

Three ways to choose variants, all driven through the C ABI:
  * exhaustive search per query (the reference for pick quality);
  * Algorithm 1 over a whole workload: one variant for all its queries of a
    kind, as the paper's feature-wise learning does per processor;
  * the learned cost model: trained on timings of sampled variants of other
    queries, it predicts every variant of a query and picks the fastest.

The mixed workload (C5) reads windows of shared column pools; `register_c5`
puts the pools on the device once and registers each window as a table of
views into them.
"""
from __future__ import annotations

import math

import numpy as np

from . import hawk


def register_c5(ctx, pools: dict, queries: list, prefix: str = "") -> list:
    """Registers the pools' dimension tables and each query's window; returns query handles
    (with the query's selectivity as its catalog statistic)."""
    import torch
    dev = {p: {c: torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for c, a in cols.items()}
           for p, cols in pools.items()}
    ctx._keep.append(dev)
    for j in range(4):
        name = f"d{j}"
        if name not in ctx.tables:
            ctx.register(name, dev[name])
    handles = []
    for q in queries:
        win = prefix + q["window"]
        spec = dict(q["spec"])
        spec["main"] = dict(spec["main"], table=win)
        o, n = q["offset"], q["rows"]
        ctx.register(win, {c: t[o:o + n] for c, t in dev[q["pool"]].items()})
        h = hawk.build_query(ctx, spec)
        h.set_stats(q["selectivity"])
        handles.append(h)
    return handles


def timed(ctx, q, v, reps: int, limit_ms: float) -> float:
    """Median time of (q, v); +inf when the variant is pruned (Section 9.1) or infeasible."""
    try:
        return hawk.time_variant(ctx, q, v, reps=reps, limit_ms=limit_ms)
    except hawk.HawkError as e:
        if e.code in (hawk.HAWK_E_TIMEOUT, hawk.HAWK_E_INFEASIBLE):
            return math.inf
        raise


def variant_key(q, v) -> str:
    """Variant identity within q's space (hash-table dimensions vanish without a table)."""
    space = hawk.variant_space(q)
    tabled = any(x.ht or x.hash for x in space)
    if not tabled:
        v = hawk.hawk_variant(v.proj_strategy, v.mem, v.pred, 0, 0, v.agg_strategy, v.reserved0, v.reserved1,
                              v.thread_mult, v.wg_size)
    return hawk.format_variant(v)


class Ensemble:
    """Cost models trained on the same timings from different seeds; picks by the
    members' mean predicted ln(ms) plus `penalty` standard deviations (their
    disagreement marks predictions far from the training timings)."""

    def __init__(self, ctx, size: int = 5, penalty: float = 1.0, seed: int = 1):
        self.models = [hawk.Model(ctx, seed=seed + k) for k in range(size)]
        self.penalty = penalty

    def train(self, X, y, epochs=300, batch=512, lr=3e-3, seed=2) -> float:
        """Trains every member; returns the members' mean training MSE."""
        return float(np.mean([m.train(X, y, epochs=epochs, batch=batch, lr=lr, seed=seed + 7919 * k)
                              for k, m in enumerate(self.models)]))

    def pick(self, queries: list):
        return hawk.model_pick_ensemble(self.models, self.penalty, queries)

    def free(self):
        for m in self.models:
            m.free()


def training_set(ctx, queries: list, per_query: int, reps: int, limit_ms: float, seed: int, progress=None):
    """Features and ln(ms) of up to `per_query` sampled variants of each query.
    A pruned variant enters with the limit as its time."""
    rng = np.random.default_rng(seed)
    X, y = [], []
    for n, q in enumerate(queries):
        if progress:
            progress(f"training timings: query {n + 1}/{len(queries)}")
        space = hawk.variant_space(q)
        idx = rng.choice(len(space), size=min(per_query, len(space)), replace=False)
        for i in sorted(idx):
            ms = timed(ctx, q, space[i], reps, limit_ms)
            X.append(q.features(space[i]))
            y.append(math.log(min(ms, limit_ms)))
    return np.asarray(X, np.float32), np.asarray(y, np.float32)


def exhaustive(ctx, q, reps: int, limit_ms: float) -> dict:
    """Time of every variant of q's space, keyed by variant_key."""
    return {variant_key(q, v): timed(ctx, q, v, reps, limit_ms) for v in hawk.variant_space(q)}


def alg1_per_kind(ctx, queries: list, reps: int, limit_ms: float, max_iters: int = 5) -> dict:
    """Algorithm 1 over each kind's sub-workload: {kind: (variant, report)}."""
    out = {}
    for kind in sorted({q.kind for q in queries}):
        W = [q for q in queries if q.kind == kind]
        v, rep = hawk.explore(ctx, W, hawk.HAWK_EXPLORE_FEATURE_WISE, reps=reps, max_iters=max_iters,
                              limit_ms=limit_ms)
        out[kind] = (v, rep)
    return out


def pick_quality(ctx, queries: list, model, reps: int, limit_ms: float, alg1: dict | None = None,
                 progress=None, extra: dict | None = None) -> dict:
    """Runtime of the model's per-query picks and of Algorithm 1's per-workload variant,
    relative to each query's exhaustive best: r_q = t(pick_q) / t(best_q). `extra`
    names further pickers (objects with .pick(queries)) scored on the same search."""
    if alg1 is None:
        alg1 = alg1_per_kind(ctx, queries, reps, limit_ms)
    pickers = {"model": model, **(extra or {})}
    picks = {name: p.pick(queries)[0] for name, p in pickers.items()}
    rows = []
    for n, q in enumerate(queries):
        if progress:
            progress(f"exhaustive search: query {n + 1}/{len(queries)}")
        table = exhaustive(ctx, q, reps, limit_ms)
        best_key = min(table, key=table.get)
        row = {"best_ms": table[best_key], "best": best_key}
        chosen = {name: pv[n] for name, pv in picks.items()}
        chosen["alg1"] = alg1[q.kind][0]
        for name, v in chosen.items():
            t = table.get(variant_key(q, v))
            if t is None:
                t = timed(ctx, q, v, reps, limit_ms)
            key = "pick" if name == "model" else name
            row[key + "_ms"] = t
            row[key] = variant_key(q, v)
        rows.append(row)

    def ratios(k):
        return np.array([r[k] / r["best_ms"] for r in rows])

    out = {"queries": len(rows)}
    for name in list(pickers) + ["alg1"]:
        k = ("pick" if name == "model" else name) + "_ms"
        r = ratios(k)
        finite = np.isfinite(r)
        out[name] = {"geomean_ratio": float(np.exp(np.mean(np.log(r[finite])))) if finite.any() else math.inf,
                     "total_ratio": float(sum(x[k] for x in rows) / sum(x["best_ms"] for x in rows)),
                     "max_ratio": float(np.max(r)), "pruned_picks": int((~finite).sum())}
    out["per_query"] = rows
    return out
