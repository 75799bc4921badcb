"""Host checks of the benchmark script: the one-GPU contract and its per-kernel-class tables."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                         capture_output=True, text=True, timeout=300)
    assert out.returncode != 0
    assert "one GPU" in out.stderr and out.stdout.strip() == ""


def test_work_tables_name_library_kernel_classes():
    """Every class the roofline tables price is one the library counts work for."""
    binding = pytest.importorskip("paper_1112_1710_amd.binding")
    try:
        binding.load_library()
    except ImportError as e:
        pytest.skip(str(e))
    import bench
    from workloads import hierarchies as H
    classes = set(binding.Hierarchy(H.small_two_level(), device=None).step_work())
    assert set(bench.ALU_BOUND) <= classes
    assert set(bench.WORDS_PER_UNIT) <= classes
    assert all(v > 0 for v in bench.WORDS_PER_UNIT.values())
    h = bench.sources_hash()
    assert len(h.split(":")) == 2 and all(len(x) == 16 for x in h.split(":"))


def test_cpu_baseline_sample_runs_the_oracle_on_the_workload():
    """The oracle's host baseline: a seeded sample of the workload's own patches, one core and a pool."""
    import bench
    out = bench.cpu_baseline("uniform32", 1)
    assert out["kind"] == "oracle" and out["unit"] == "zone-updates/s"
    assert out["value"] > 0 and out["single_core"]["value"] > 0 and out["cores"] >= 1
    assert "CPU:" in out["sample"]


def test_measured_traffic_applies_only_to_its_sources_and_fused_levels(monkeypatch):
    """A stored HBM reading is reported only for the kernel sources it was taken on and for a run that
    fused the same levels (the launches its per-launch average runs over)."""
    import bench
    monkeypatch.setattr(bench, "MEASURED_TRAFFIC", {("deep", "fp32", "primhalf"): [
        {"bytes_per_launch": 1.0, "fused_levels": [4, 5], "sources": bench.sources_hash()},
        {"bytes_per_launch": 2.0, "fused_levels": [3, 4, 5], "sources": bench.sources_hash()},
        {"bytes_per_launch": 3.0, "fused_levels": [5], "sources": "0" * 16 + ":" + "0" * 16}]})
    assert bench.measured_traffic("deep", "fp32", "primhalf", {4, 5})["bytes_per_launch"] == 1.0
    assert bench.measured_traffic("deep", "fp32", "primhalf", {5, 4, 3})["bytes_per_launch"] == 2.0
    assert bench.measured_traffic("deep", "fp32", "primhalf", {5}) is None           # other sources
    assert bench.measured_traffic("deep", "fp32", "primhalf", {2, 3, 4, 5}) is None  # no reading
    assert bench.measured_traffic("deep", "fp32_mixed", "primhalf", {4, 5}) is None
    assert bench.measured_traffic("two_level", "fp32", "flux", set()) is None


def test_stored_readings_match_the_current_kernel_sources():
    """The committed counter readings were taken on the kernel sources in the tree."""
    import bench
    for recs in bench.MEASURED_TRAFFIC.values():
        assert all(r["sources"] == bench.sources_hash() for r in recs)
    assert all(r["sources"] == bench.sources_hash() for r in bench.MEASURED_VALU_ISSUE.values())
