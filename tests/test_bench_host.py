"""Host logic of bench.py, on the CPU: the single-GPU contract and the rule
that a committed counter summary supplies HBM traffic only while the
kernel's sources are the ones it was taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""  # no bench line


@pytest.mark.parametrize("workload,kernel", sorted(bench.TRAFFIC_PROFILES))
def test_traffic_is_dropped_once_the_kernel_sources_change(monkeypatch, workload, kernel):
    name = bench.TRAFFIC_PROFILES[(workload, kernel)]
    assert os.path.exists(os.path.join(ROOT, "profiles", name)), name
    # another set of sources hashes differently: the summary no longer applies
    changed = dict(bench.KERNEL_SOURCES)
    changed[kernel] = tuple(bench.KERNEL_SOURCES[kernel]) + ("bench.py",)
    monkeypatch.setattr(bench, "KERNEL_SOURCES", changed)
    assert bench.measured_traffic(workload, kernel) is None


def test_traffic_of_an_unprofiled_kernel_is_none():
    assert bench.measured_traffic("plain", "k_group_direct") is None
    assert bench.measured_traffic("block-sparse-1.5M", "no_such_kernel") is None
