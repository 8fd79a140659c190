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


def upload_pools(ctx, pools: dict) -> dict:
    """The pools as device tensors (kept alive by the context)."""
    import torch
    dev = {p: {c: torch.from_numpy(np.ascontiguousarray(a)).to("cuda") for c, a in cols.items()}
           for p, cols in pools.items()}
    ctx._keep.append(dev)
    return dev


def register_c5(ctx, pools: dict, queries: list, prefix: str = "", dev: dict | None = None) -> list:
    """Registers the pools' dimension tables and each query's window; returns query handles
    (with the query's selectivity as its catalog statistic). `dev`: the pools
    already on the device (upload_pools), else they are uploaded here."""
    if dev is None:
        dev = upload_pools(ctx, pools)
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


def variant_key(q, v, tabled: bool | None = None) -> str:
    """Variant identity within q's space (hash-table dimensions vanish without a table)."""
    if tabled is None:
        tabled = any(x.ht or x.hash for x in hawk.variant_space(q))
    if not tabled:
        v = hawk.hawk_variant(v.proj_strategy, v.mem, v.pred, 0, 0, v.agg_strategy, v.unroll, v.filter_mode,
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

    def scores(self, q, variants: list):
        """Members' mean and standard deviation of predicted ln(ms) per variant."""
        X = np.stack([q.features(v) for v in variants])
        P = np.stack([m.predict(X) for m in self.models]).astype(np.float64)
        return P.mean(axis=0), P.std(axis=0)

    def free(self):
        for m in self.models:
            m.free()


class WithFallback:
    """Per-query picks of an ensemble over a per-workload variant: a query
    keeps `fallback[kind]` (e.g. Algorithm 1's variant for its kind) unless the
    ensemble's own pick is predicted faster at its pessimistic score (mean +
    penalty x sd of the members' ln(ms)) than the fallback at its optimistic
    one (mean - penalty x sd). Greedy search stays the fallback; the model
    departs from it only where its members agree on a gain larger than their
    spread on both variants.

    With `race_ctx`, the two candidates are instead timed on the query itself
    (`race_reps` runs each, the faster kept): the model proposes one variant,
    one short race against the per-workload variant decides. `race_ms` sums
    the time those runs took."""

    def __init__(self, ens: Ensemble, fallback: dict, race_ctx=None, race_reps: int = 2):
        self.ens = ens
        self.fallback = fallback
        self.race_ctx = race_ctx
        self.race_reps = race_reps
        self.race_ms = 0.0
        self._raced = {}  # id(query) -> (query, the race's winner); the query kept alive with its id

    def pick(self, queries: list):
        picks, _ = self.ens.pick(queries)
        out = []
        for q, v in zip(queries, picks):
            if self.race_ctx is not None and id(q) in self._raced:
                out.append(self._raced[id(q)][1])
                continue
            fb = self.fallback.get(q.kind)
            if fb is None or variant_key(q, v) == variant_key(q, fb):
                out.append(v if fb is None else fb)
                continue
            if self.race_ctx is not None:
                t = [timed(self.race_ctx, q, x, self.race_reps, 0.0) for x in (v, fb)]
                self.race_ms += self.race_reps * sum(x for x in t if math.isfinite(x))
                out.append(v if t[0] < t[1] else fb)
                self._raced[id(q)] = (q, out[-1])
                continue
            mean, sd = self.ens.scores(q, [v, fb])
            out.append(v if mean[0] + self.ens.penalty * sd[0] < mean[1] - self.ens.penalty * sd[1] else fb)
        return out, None


# a variant that is fast for most pipelines of a kind: the reference of the
# relative pruning limit of the training timings
REFERENCE = {1: dict(proj_strategy=1, mem=1, pred=0, thread_mult=1024, wg_size=256),
             2: dict(proj_strategy=1, mem=1, pred=0, ht=0, hash=1, agg_strategy=0, thread_mult=8, wg_size=256)}


def training_set(ctx, queries: list, per_query: int, reps: int, limit_ms: float, seed: int, progress=None,
                 factor: float | None = None):
    """Features and ln(ms) of up to `per_query` sampled variants of each query.
    A pruned variant enters with its limit as its time. With `factor` the
    limit of a query is min(limit_ms, factor x its reference variant's time)."""
    rng = np.random.default_rng(seed)
    X, y = [], []
    for n, q in enumerate(queries):
        if progress:
            progress(f"training timings: query {n + 1}/{len(queries)}")
        space = hawk.variant_space(q)
        lim = limit_ms
        if factor is not None:
            ref = timed(ctx, q, hawk.variant(**REFERENCE[q.kind]), reps, limit_ms)
            if math.isfinite(ref):
                lim = min(limit_ms, factor * ref)
        idx = rng.choice(len(space), size=min(per_query, len(space)), replace=False)
        for i in sorted(idx):
            ms = timed(ctx, q, space[i], reps, lim)
            X.append(q.features(space[i]))
            y.append(math.log(min(ms, lim)))
    return np.asarray(X, np.float32), np.asarray(y, np.float32)


def ranked(ens, q, k: int) -> list:
    """The k variants of q's space with the lowest ensemble score (mean +
    penalty x standard deviation of the members' predicted ln(ms)), best first."""
    space = hawk.variant_space(q)
    X = np.stack([q.features(v) for v in space])
    P = np.stack([m.predict(X) for m in ens.models]).astype(np.float64)
    score = P.mean(axis=0) + ens.penalty * P.std(axis=0)
    return [space[i] for i in np.argsort(score, kind="stable")[:k]]


def refine(ctx, queries: list, ens, X, y, top: int, rounds: int, reps: int, limit_ms: float,
           factor: float | None = None, progress=None, **train_kw):
    """Active sampling: times each training query's `top` best-ranked
    variants under the current ensemble, adds them to the training set and
    retrains, `rounds` times. A model that ranks a slow variant first learns
    its real time here, where one-off sampling rarely reaches. Returns the
    grown training set."""
    for r in range(rounds):
        nx, ny = [], []
        for n, q in enumerate(queries):
            if progress and n % 16 == 0:
                progress(f"active sampling round {r + 1}: query {n + 1}/{len(queries)}")
            lim = limit_ms
            if factor is not None:
                ref = timed(ctx, q, hawk.variant(**REFERENCE[q.kind]), reps, limit_ms)
                if math.isfinite(ref):
                    lim = min(limit_ms, factor * ref)
            for v in ranked(ens, q, top):
                ms = timed(ctx, q, v, reps, lim)
                nx.append(q.features(v))
                ny.append(math.log(min(ms, lim)))
        X = np.concatenate([X, np.asarray(nx, np.float32)])
        y = np.concatenate([y, np.asarray(ny, np.float32)])
        ens.train(X, y, **train_kw)
    return X, y


def exhaustive(ctx, q, reps: int, limit_ms: float, factor: float | None = None, first=()) -> dict:
    """Time of every variant of q's space, keyed by variant_key. With `factor`,
    the pruning limit follows the search: a variant slower than `factor` times
    the fastest one measured so far (and than limit_ms) counts as +inf (the
    pruning rule of Section 9.1, relative to the running best). The variants in
    `first` are measured first, under limit_ms only."""
    out = {}
    best = math.inf
    space = hawk.variant_space(q)
    tabled = any(x.ht or x.hash for x in space)
    first_keys = {variant_key(q, f, tabled) for f in first}
    for v in list(first) + list(space):
        key = variant_key(q, v, tabled)
        if key in out:
            continue
        lim = limit_ms if factor is None or not math.isfinite(best) or key in first_keys \
            else min(limit_ms, factor * best)
        t = timed(ctx, q, v, reps, lim)
        out[key] = t
        best = min(best, t)
    return out


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
                 progress=None, extra: dict | None = None, factor: float | None = None,
                 deadline: float | None = None, confirm_reps: int = 0) -> dict:
    """Runtime of the model's per-query picks and of Algorithm 1's per-workload variant,
    relative to each query's exhaustive best: r_q = t(pick_q) / t(best_q). `extra`
    names further pickers (objects with .pick(queries)) scored on the same search.
    `factor`: prune relative to the running best (the picks are measured first);
    `deadline` (time.perf_counter() value): stop after the query that passes it.
    `confirm_reps` > 0: the search's best variant and every picked variant are
    timed again with that many runs each, and those times are compared (the
    best is the fastest of them). The minimum over hundreds of short, noisy
    medians is biased low; timing the finalists alike removes that bias from
    the ratios."""
    import time
    if alg1 is None:
        alg1 = alg1_per_kind(ctx, queries, reps, limit_ms)
    pickers = {"model": model, **(extra or {})}
    picks = {name: p.pick(queries)[0] for name, p in pickers.items()}
    rows = []
    for n, q in enumerate(queries):
        if deadline is not None and time.perf_counter() > deadline:
            break
        if progress:
            progress(f"exhaustive search: query {n + 1}/{len(queries)}")
        first = [pv[n] for pv in picks.values()] + [alg1[q.kind][0]]
        table = exhaustive(ctx, q, reps, limit_ms, factor=factor, first=first)
        best_key = min(table, key=table.get)
        chosen = {name: pv[n] for name, pv in picks.items()}
        chosen["alg1"] = alg1[q.kind][0]
        if confirm_reps > 0:
            space = hawk.variant_space(q)
            tabled = any(x.ht or x.hash for x in space)
            finalists = {variant_key(q, v, tabled): v for v in chosen.values()}
            finalists.setdefault(best_key, next(v for v in space if variant_key(q, v, tabled) == best_key))
            for key, v in finalists.items():
                if math.isfinite(table.get(key, math.inf)):
                    table[key] = timed(ctx, q, v, confirm_reps, limit_ms)
            best_key = min(finalists, key=lambda k_: table.get(k_, math.inf))
        row = {"best_ms": table[best_key], "best": best_key}
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

    out = {"queries": len(rows), "queries_planned": len(queries)}
    for name in list(pickers) + ["alg1"]:
        k = ("pick" if name == "model" else name) + "_ms"
        r = ratios(k)
        finite = np.isfinite(r)
        out[name] = {"geomean_ratio": float(np.exp(np.mean(np.log(r[finite])))) if finite.any() else math.inf,
                     "total_ratio": float(sum(x[k] for x in rows) / sum(x["best_ms"] for x in rows)),
                     "max_ratio": float(np.max(r)), "pruned_picks": int((~finite).sum())}
    out["per_query"] = rows
    return out
