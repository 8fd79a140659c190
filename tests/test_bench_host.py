"""Host logic of bench.py (no GPU): the measured-traffic table is reported
only while the kernel sources and the pipeline's variant are the ones it was
measured on, and the algorithmic byte counts of the mixed workload."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_entries_well_formed(bench):
    for name, t in bench.TRAFFIC.items():
        assert name in bench.DEFAULT_VARIANTS
        assert set(t) == {"sources_sha", "variant_sha", "per_kernel", "total"}
        assert len(t["sources_sha"]) == 16 and len(t["variant_sha"]) == 16
        assert t["total"] == pytest.approx(sum(t["per_kernel"].values()))
        assert all(k in bench.KERNEL_FAMILIES for k in t["per_kernel"])


def test_traffic_only_for_the_measured_sources_and_variant(bench, monkeypatch):
    entry = {"sources_sha": bench.kernel_sources_sha(), "variant_sha": bench.variant_sha("c2z"),
             "per_kernel": {"k_agg": 9.0e8, "k_spill_agg": 3.0e8}, "total": 1.2e9}
    monkeypatch.setattr(bench, "TRAFFIC", {"c2z": entry})
    assert bench.traffic_for("c2z") == entry
    assert bench.traffic_for("c2u") is None
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda: "0" * 16)
    assert bench.traffic_for("c2z") is None
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda: entry["sources_sha"])
    changed = {k: dict(v) for k, v in bench.DEFAULT_VARIANTS.items()}
    changed["c2z"]["wg_size"] = 512
    monkeypatch.setattr(bench, "DEFAULT_VARIANTS", changed)
    assert bench.traffic_for("c2z") is None


def test_c5_algorithmic_bytes(bench):
    # projection: 4 B per row + 20 B per qualifying row
    assert bench.c5_algo_bytes({"kind": 1, "rows": 1000, "selectivity": 0.5}) == pytest.approx(1000 * (4 + 10))
    # aggregation: 4 B per row + 12 B per qualifying row
    assert bench.c5_algo_bytes({"kind": 2, "rows": 1000, "selectivity": 0.25}) == pytest.approx(1000 * (4 + 3))
    # star join, all rows joining: four keys and the revenue for every row = 24 B
    assert bench.c5_algo_bytes({"kind": 3, "rows": 1000, "selectivity": 1.0}) == pytest.approx(24_000)
    # per-dimension selectivity 1/2: keys 4 (1 + 1/2 + 1/4 + 1/8) + revenue 8/16
    assert bench.c5_algo_bytes({"kind": 3, "rows": 16, "selectivity": 1 / 16}) == pytest.approx(16 * (7.5 + 0.5))


def test_every_timed_pipeline_has_bytes_and_a_variant(bench):
    for w, names in bench.WORKLOADS.items():
        for n in names:
            assert n in bench.DEFAULT_VARIANTS and n in bench.ALGO_BYTES_PER_ROW
    assert bench.HEADLINE["all"] == "c4"


def test_same_answer_catches_any_difference(bench):
    """The check of the device's answer on the baseline sample: equal
    answers pass, a changed count, key, sum or AVG beyond 1e-12 fails."""
    import copy
    import oracle
    tables, spec = bench.make_pipeline("c4", rows=5000)
    ref = oracle.run(tables, spec)
    assert bench.same_answer(copy.deepcopy(ref), ref)
    for mutate in (lambda a: a["count"].__setitem__(0, a["count"][0] + 1),
                   lambda a: a["keys"][0].__setitem__(0, a["keys"][0][0] + 7),
                   lambda a: a["aggs"][1].__setitem__(0, a["aggs"][1][0] + 1),
                   lambda a: a["aggs"][7].__setitem__(0, a["aggs"][7][0] * (1 + 1e-9))):
        got = copy.deepcopy(ref)
        mutate(got)
        assert not bench.same_answer(got, ref)
    tables, spec = bench.make_pipeline("c1", rows=5000)
    ref = oracle.run(tables, spec)
    got = copy.deepcopy(ref)
    assert bench.same_answer(got, ref)
    got["cols"][0][3] += 1
    assert not bench.same_answer(got, ref)
