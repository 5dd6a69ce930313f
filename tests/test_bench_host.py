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


@pytest.mark.parametrize("kernel", sorted(bench.KERNEL_SOURCES))
def test_traffic_needs_matching_sources_and_instance(tmp_path, monkeypatch, kernel):
    monkeypatch.setattr(bench, "traffic_file", lambda k: str(tmp_path / ("%s.md" % k)))
    f = tmp_path / ("%s.md" % kernel)
    sha = bench.kernel_sources_sha256(kernel)
    _write(f, sha, "abc")
    assert bench.measured_traffic("abc", kernel) == pytest.approx(1.5e9)
    assert bench.measured_traffic("abd", kernel) is None          # another instance
    _write(f, "0" * 64, "abc")
    assert bench.measured_traffic("abc", kernel) is None          # other kernel sources
    _write(f, sha, "abc", value="n/a")
    assert bench.measured_traffic("abc", kernel) is None          # unreadable figure
    f.unlink()
    assert bench.measured_traffic("abc", kernel) is None          # no summary


def test_elmore_and_dp_sources_differ():
    assert bench.kernel_sources_sha256("k_batched_dp") != bench.kernel_sources_sha256("k_elmore_wave")


@pytest.mark.parametrize("kernel", sorted(bench.KERNEL_SOURCES))
def test_committed_traffic_summary_names_sources_and_instance(kernel):
    vals = {}
    with open(bench.traffic_file(kernel)) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("|", "#", "`")):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    assert float(vals["traffic_bytes_per_launch"]) > 0
    assert len(vals["kernel_sources_sha256"]) == 64 and len(vals["workload_digest"]) == 64
