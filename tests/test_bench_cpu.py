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
