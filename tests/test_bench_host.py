"""Host logic of bench.py (no GPU): the measured-traffic table is reported
only while the kernel sources and the workload's variants are the ones it
was measured on."""
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
    assert bench.TRAFFIC, "no measured traffic"
    for (kernel, workload), t in bench.TRAFFIC.items():
        assert workload in bench.WORKLOADS and kernel == "k_agg"
        assert set(t) == {"sources_sha", "variants_sha", "bytes_per_launch"}
        assert t["bytes_per_launch"] > 0 and len(t["sources_sha"]) == 16 and len(t["variants_sha"]) == 16


def test_traffic_only_for_the_measured_sources_and_variants(bench, monkeypatch):
    (kernel, workload), t = next(iter(bench.TRAFFIC.items()))
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda k: t["sources_sha"])
    monkeypatch.setattr(bench, "variants_sha", lambda w: t["variants_sha"])
    assert bench.traffic_for(kernel, workload) == t["bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda k: "0" * 16)
    assert bench.traffic_for(kernel, workload) is None
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda k: t["sources_sha"])
    monkeypatch.setattr(bench, "variants_sha", lambda w: "f" * 16)
    assert bench.traffic_for(kernel, workload) is None
    assert bench.traffic_for("k_other", workload) is None


def test_variants_sha_follows_the_default_variants(bench, monkeypatch):
    before = bench.variants_sha("c2")
    changed = {k: dict(v) for k, v in bench.DEFAULT_VARIANTS.items()}
    changed["c2z"]["wg_size"] = 512
    monkeypatch.setattr(bench, "DEFAULT_VARIANTS", changed)
    assert bench.variants_sha("c2") != before
