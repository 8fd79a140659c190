"""Helpers of the GPU parity tests: run a query through the C ABI and compare
with the oracle's answer element by element."""
from __future__ import annotations

import sys
from fractions import Fraction

import numpy as np

import oracle
from paper_1709_00700_amd import hawk

AVG_RTOL = Fraction(1, 10**12)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare(got: dict, ref: dict, spec: dict, label: str = ""):
    assert got["rows"] == ref["rows"], (label, got["rows"], ref["rows"])
    if ref["kind"] == "project":
        for c, (g, r) in enumerate(zip(got["cols"], ref["cols"])):
            if not np.array_equal(g, r):
                bad = np.nonzero(g != r)[0][:5]
                raise AssertionError(f"{label}: column {c} differs at rows {bad.tolist()}: "
                                     f"{g[bad].tolist()} vs {r[bad].tolist()}")
        return
    for j, (g, r) in enumerate(zip(got["keys"], ref["keys"])):
        assert np.array_equal(g, r), (label, "group key", j)
    assert np.array_equal(got["count"], ref["count"]), (label, "count")
    for j, (fn, _, wide) in enumerate(spec["main"]["aggs"]):
        g, r = got["aggs"][j], ref["aggs"][j]
        if fn == "avg":
            for x, y in zip(g, r):
                if y != y:
                    assert x != x
                    continue
                ex = Fraction(float(y))  # oracle AVG is the double of the exact quotient
                assert abs(Fraction(float(x)) - ex) <= AVG_RTOL * abs(ex) + Fraction(1, 10**300), (label, "avg", x, y)
        elif wide:
            assert [int(x) for x in g] == [int(x) for x in r], (label, "wide sum", j)
        else:
            assert np.array_equal(np.asarray(g, dtype=np.int64), np.asarray(r, dtype=np.int64)), (label, fn, j)


def run_variants(ctx, tables, spec, variants, ref=None, label=""):
    """Registers `tables`, builds the query and checks every variant against the oracle."""
    if ref is None:
        ref = oracle.run(tables, spec)
    ctx.register_numpy(tables)
    q = hawk.build_query(ctx, spec)
    for v in variants:
        r = hawk.execute(ctx, q, v)
        got = r.to_numpy(spec)
        r.free()
        compare(got, ref, spec, f"{label} {hawk.format_variant(v)}")
    return q, ref


def sample(variants, k, seed=0):
    if len(variants) <= k:
        return variants
    rng = np.random.default_rng(seed)
    idx = sorted(rng.choice(len(variants), size=k, replace=False))
    return [variants[i] for i in idx]
