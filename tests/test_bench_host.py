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


def _write_csv(path, header, rows):
    import csv
    with open(path, "w", newline="") as fh:
        wr = csv.writer(fh)
        wr.writerow(header)
        wr.writerows(rows)


def test_profile_summary_scales_counters_by_the_copy(monkeypatch, tmp_path):
    """summarize_profile: per-launch means of FETCH_SIZE / WRITE_SIZE (KiB) scaled so that
    the largest plain device copy reads 1 GiB each way; the written block is what
    profiled_traffic reads back."""
    for d in ("trace", "fetch", "write"):
        (tmp_path / d).mkdir()
    _write_csv(tmp_path / "trace" / "x_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
               [["void sem::k_ax_helm<8, double, 1, false>(sem::AxArgs<double>, sem::DEo<8, double>)", 2, 400000,
                 200000, 60.0],
                ["__amd_rocclr_copyBuffer", 1, 300000, 300000, 40.0]])
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Grid_Size"]
    # the reference is the first copy of the largest grid (dispatch 2); a later copy of
    # the same grid (dispatch 9, partly served from cache) must not be taken
    _write_csv(tmp_path / "fetch" / "x_counter_collection.csv", hdr,
               [[5, "void sem::k_ax_helm<8, double, 1, false>(sem::AxArgs<double>, sem::DEo<8, double>)",
                 "FETCH_SIZE", 1000.0, 4096],
                [6, "void sem::k_ax_helm<8, double, 1, false>(sem::AxArgs<double>, sem::DEo<8, double>)",
                 "FETCH_SIZE", 3000.0, 4096],
                [9, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 100000.0, 131072],
                [2, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0, 131072],
                [1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 10.0, 64]])
    _write_csv(tmp_path / "write" / "x_counter_collection.csv", hdr,
               [[5, "void sem::k_ax_helm<8, double, 1, false>(sem::AxArgs<double>, sem::DEo<8, double>)",
                 "WRITE_SIZE", 500.0, 4096],
                [2, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0, 131072]])
    out = tmp_path / "s.md"
    bench.summarize_profile(str(tmp_path / "trace"), str(tmp_path / "fetch"), str(tmp_path / "write"), str(out),
                            "test", "workload", ["cmd"], ["bench.py"])
    monkeypatch.setattr(bench, "PROFILE_MD", str(out))
    # fetch: mean 2000 KiB x 2 (the copy read 512 MiB for 1 GiB moved); write: 500 KiB x 1
    assert bench.profiled_traffic("sem::k_ax_helm<8, double, 1, false>") == 2000 * 1024 * 2 + 500 * 1024
    text = out.read_text()
    assert "| `sem::k_ax_helm<8, double, 1, false>` | 2 | 200.00 |" in text
