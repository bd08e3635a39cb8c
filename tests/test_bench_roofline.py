"""Host-side checks of the benchmark's roofline record (no GPU): frac is
the counter-measured DRAM bytes per launch over the launch duration against
8 TB/s, the logical bytes stay in a separate field, stale counter summaries
give no DRAM figure, and the compulsory floor follows its definition."""
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture
def bench(monkeypatch, tmp_path):
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(mod, "ROOT", str(tmp_path))
    return mod, tmp_path


def write_summary(tmp_path, kernel, workload, rec):
    text = f"# summary\n\n```json\n{json.dumps(rec)}\n```\n"
    (tmp_path / "profiles" / f"{kernel}_{workload}_hbm_traffic.md").write_text(text)


def test_frac_is_dram_bytes_over_time_against_peak(bench, monkeypatch):
    mod, tmp = bench
    monkeypatch.setattr(mod, "kernel_source_sha", lambda: "abc")
    write_summary(tmp, "gather", "colour", {"kernel_source_sha": "abc", "hbm_bytes_per_launch": 1.2e9,
                                            "td_busy": 0.7})
    r = mod.roofline_record("gather", 0.8e-3, 96 * 116_000_000, 116_000_000, "colour", 20, {}, floor=3.2e8)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(1.2e9 / 0.8e-3 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(1.2e9 / 0.8e-3 / 1e9 / 8000.0, rel=1e-3)
    assert r["traffic"] == 1.2e9
    # the logical (algorithmic) rate is reported beside, never as frac
    assert r["algorithmic"]["GBs"] == pytest.approx(96 * 116_000_000 / 0.8e-3 / 1e9, rel=1e-3)
    assert r["algorithmic"]["bytes_per_sample"] == 96
    assert r["onchip"]["busy"] == 0.7 and r["onchip"]["peak"] == 1.0
    assert r["traffic_over_floor"] == pytest.approx(1.2e9 / 3.2e8, rel=1e-3)


def test_stale_or_missing_counters_give_no_dram_figure(bench, monkeypatch):
    mod, tmp = bench
    monkeypatch.setattr(mod, "kernel_source_sha", lambda: "new")
    write_summary(tmp, "render", "colour", {"kernel_source_sha": "old", "hbm_bytes_per_launch": 1e9})
    for k in ("render", "gather"):
        r = mod.roofline_record(k, 1e-3, 10**9, 10**7, "colour", 1, {})
        assert r["achieved"] is None and r["frac"] is None and r["traffic"] is None
        assert r["algorithmic"]["GBs"] == pytest.approx(1000.0)


def test_compulsory_floor():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod2", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    n = 128 ** 3
    # packed RGB + extinction read once per view, frames once, the update written once
    assert mod.compulsory_floor(n, 3, 8, 512, 512) == 8 * n * 16 + 8 * 3 * 512 * 512 * 4 + 3 * n * 4
    assert mod.compulsory_floor(n, 1, 8, 512, 512) == 8 * n * 8 + 8 * 512 * 512 * 4 + n * 4


def test_step_spread_percentiles_over_repeats(bench, monkeypatch):
    """The spread reruns the timed steps `repeats` times, each from a fresh
    start, and reports per-step percentiles; no repeats gives no record."""
    import torch
    mod, _ = bench
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    clock = iter([0.0, 0.010, 1.0, 1.030, 2.0, 2.020])  # 10, 30, 20 ms for 10 steps each
    monkeypatch.setattr(mod.time, "perf_counter", lambda: next(clock))
    starts, calls = [], []
    rec = mod.step_spread(lambda x, k: calls.append((x, k)), lambda: starts.append(1) or "x0", 10, 3)
    assert calls == [("x0", 10)] * 3 and len(starts) == 3
    assert rec["repeats"] == 3 and rec["steps_each"] == 10
    assert rec["p50"] == pytest.approx(2.0)
    assert rec["p5"] == pytest.approx(1.0 + 0.1 * 1.0) and rec["p95"] == pytest.approx(3.0 - 0.1 * 1.0)
    assert mod.step_spread(None, None, 10, 0) is None


def test_max_rel_is_relative_to_the_reference_maximum(bench):
    mod, _ = bench
    assert mod.max_rel([1.0, 2.0], [1.0, 2.0]) == 0.0
    assert mod.max_rel([1.0, 2.5], [1.0, -2.0]) == pytest.approx(4.5 / 2.0)
    assert mod.max_rel([1.0], [0.0]) == 0.0
