"""Host-side checks of bench.py (no GPU): the one-GPU guard and the reader of the
committed rocprofv3 counter summary."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_profiled_traffic_unknown_kernel_and_missing_summary(monkeypatch, tmp_path):
    assert bench.profiled_traffic("no_such_kernel") is None
    monkeypatch.setattr(bench, "PROFILE_MD", str(tmp_path / "missing.md"))
    assert bench.profiled_traffic("sem::k_ax_helm<8, double, 1, false>") is None


def test_profiled_traffic_is_none_when_sources_changed(monkeypatch, tmp_path):
    """A summary whose recorded source hash does not match the sources gives None."""
    md = tmp_path / "p.md"
    md.write_text('text\n```json\n{"sources": ["bench.py"], "source_sha256": "0", '
                  '"kernels": {"k": {"fetch_bytes": 1, "write_bytes": 2}}}\n```\n')
    monkeypatch.setattr(bench, "PROFILE_MD", str(md))
    assert bench.profiled_traffic("k") is None


def test_profiled_traffic_sums_fetch_and_write_when_sources_match(monkeypatch, tmp_path):
    import hashlib
    h = hashlib.sha256(open(os.path.join(ROOT, "bench.py"), "rb").read()).hexdigest()
    md = tmp_path / "p.md"
    md.write_text('text\n```json\n{"sources": ["bench.py"], "source_sha256": "%s", '
                  '"kernels": {"k": {"fetch_bytes": 1000, "write_bytes": 24}}}\n```\n' % h)
    monkeypatch.setattr(bench, "PROFILE_MD", str(md))
    assert bench.profiled_traffic("k") == 1024
    assert bench.profiled_traffic("other") is None
