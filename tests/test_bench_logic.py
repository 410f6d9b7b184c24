"""Host-side pieces of bench.py, on the CPU: the one-GPU guard, the
algorithmic counts the roofline divides by, and the rule that the counter
traffic is reported only for the stage-kernel sources it was measured on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def test_algorithmic_flops_per_node_stage():
    """The method's count: per axis one new first difference (2), one WENO
    window (49) and two blends (26 each), p-bar 2 and LF 4: 109; three axes,
    the relative-Dubins Hamiltonian 17, the sign 1 and the RK blend averaged
    over the three stages (13/3).  The per-node kernel executes six
    differences and both windows per axis: 168 per axis."""
    assert bench.WENO_WINDOW_FLOPS == 49 and bench.WENO_BLEND_FLOPS == 26
    assert bench.weno5_flops_per_node_stage(3) == pytest.approx(3 * 109 + 17 + 1 + 13 / 3)
    assert bench.weno5_flops_per_node_stage(3, executed=True) == pytest.approx(
        3 * 168 + 17 + 1 + 13 / 3)


def test_algorithmic_bytes_per_node_stage():
    # stage 1: V in, A out; stage 2: A, V in, B out; stage 3: B, V (, V0) in, V out
    assert bench.bytes_per_node_stage(8, True) == pytest.approx(8 * 9 / 3)
    assert bench.bytes_per_node_stage(4, False) == pytest.approx(4 * 8 / 3)


def test_traffic_only_for_the_measured_sources(monkeypatch):
    m = bench.MEASURED_TRAFFIC["fp64"]
    monkeypatch.setattr(bench, "source_hash", lambda: m["src_hash"])
    want = 1024.0 * (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"])
    assert bench.measured_traffic("fp64") == pytest.approx(want)
    monkeypatch.setattr(bench, "source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("fp64") is None
    assert bench.measured_traffic("fp16") is None


def test_source_hash_follows_the_stage_sources():
    h = bench.source_hash()
    assert len(h) == 16 and h == bench.source_hash()
    for name in bench.STAGE_KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_2507_11542_amd", "csrc", name))
