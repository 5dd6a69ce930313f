"""Host logic of bench.py that needs no GPU: the one-GPU guard and the rule that a measured
traffic figure is reported only for the kernel sources and the instance it was measured on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _write(path, sha, digest, value="1.5e+09"):
    path.write_text("# summary\n\n| a | b |\n\ntraffic_bytes_per_launch: %s\nkernel_sources_sha256: %s\n"
                    "workload_digest: %s\n" % (value, sha, digest))


def test_traffic_needs_matching_sources_and_instance(tmp_path, monkeypatch):
    f = tmp_path / "traffic.md"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    sha = bench.kernel_sources_sha256()
    _write(f, sha, "abc")
    assert bench.measured_traffic("abc") == pytest.approx(1.5e9)
    assert bench.measured_traffic("abd") is None          # another instance
    _write(f, "0" * 64, "abc")
    assert bench.measured_traffic("abc") is None          # other kernel sources
    _write(f, sha, "abc", value="n/a")
    assert bench.measured_traffic("abc") is None          # unreadable figure
    f.unlink()
    assert bench.measured_traffic("abc") is None          # no summary


def test_committed_traffic_summary_names_sources_and_instance():
    vals = {}
    with open(bench.TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("|", "#", "`")):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    assert float(vals["traffic_bytes_per_launch"]) > 0
    assert len(vals["kernel_sources_sha256"]) == 64 and len(vals["workload_digest"]) == 64
