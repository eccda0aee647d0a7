"""CPU checks of bench.py's host logic: it refuses more than one GPU, and it
reports profiler-measured figures only while the kernel sources are the ones
the committed counter runs were taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.join(os.path.dirname(__file__), "..")
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"] and msg["n_gpus"] == 2


def test_measured_figures_follow_the_source_digest(monkeypatch, tmp_path):
    rec = {"step": {"kernel_digest": bench.kernel_digest(),
                    "workloads": {"w": {"bytes_per_launch": 123, "valu_instructions_per_node_step": 7.5}}},
           "adjoint": {"kernel_digest": "0" * 16, "workloads": {"a": {"bytes_per_launch": 9}}}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("w") == 123
    assert bench.measured_traffic("w", field="valu_instructions_per_node_step") == 7.5
    assert bench.measured_traffic("missing") is None
    # a digest taken on other sources: no figure
    assert bench.measured_traffic("a", section="adjoint") is None
    monkeypatch.setattr(bench, "kernel_digest", lambda sources=None: "f" * 16)
    assert bench.measured_traffic("w") is None


def test_committed_record_is_readable():
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    for sec in ("step", "adjoint"):
        assert len(rec[sec]["kernel_digest"]) == 16
        for w in rec[sec]["workloads"].values():
            # measured HBM bytes sit at or above the algorithmic ones, up to
            # the counters' own rounding
            assert 0.999 <= w["bytes_per_launch"] / w["algorithmic_bytes"] < 1.5
