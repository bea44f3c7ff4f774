"""Host logic of the profiler summaries: the pair-kernel source hash that keys the recorded
counters, and the per-stream kernel time and overlap of a kernel trace."""
import csv
import os
import shutil

from paper_1612_00474_amd import profile_summary as ps


def _copy_sources(tmp_path):
    (tmp_path / "csrc").mkdir()
    for name in ps.PAIR_SOURCES:
        shutil.copy(os.path.join(ps.PKG, "csrc", name), tmp_path / "csrc" / name)


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    _copy_sources(tmp_path)
    monkeypatch.setattr(ps, "PKG", str(tmp_path))
    h0 = ps.kernel_source_hash()
    f = tmp_path / "csrc" / "matvec.hip"
    text = f.read_text()
    f.write_text("// a comment line\n\n" + text.replace("\n", "  // trailing comment\n", 1))
    assert ps.kernel_source_hash() == h0
    f.write_text(text + "\nstatic int unused_symbol = 1;\n")
    assert ps.kernel_source_hash() != h0


def _trace(tmp_path, rows):
    d = tmp_path / "trace"
    d.mkdir()
    keys = ["Kernel_Name", "Stream_Id", "Start_Timestamp", "End_Timestamp"]
    with open(d / "t_kernel_trace.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=keys)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(keys, r)))
    with open(d / "t_kernel_stats.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs",
                                           "MinNs", "MaxNs"])
        w.writeheader()
        w.writerow({"Name": "k", "Calls": len(rows), "TotalDurationNs": 1, "AverageNs": 1,
                    "MinNs": 1, "MaxNs": 1})
    return str(d)


def test_trace_reports_kernel_time_beside_another_stream(tmp_path, capsys):
    # stream 0: [0, 10) and [20, 30) us; stream 1: [5, 25) us.  Busy 30 us, kernel time 40 us,
    # so 10 us ran beside another kernel.
    d = _trace(tmp_path, [("a", "0", 0, 10000), ("b", "0", 20000, 30000), ("c", "1", 5000, 25000)])
    ps.trace(d, 5)
    out = capsys.readouterr().out
    assert "stream 0: 0.02, stream 1: 0.02" in out
    assert "time with at least one kernel running 0.03 ms" in out
    assert "so 0.01 ms of kernel time ran beside another kernel" in out


def test_trace_of_one_stream_has_no_overlap_line(tmp_path, capsys):
    d = _trace(tmp_path, [("a", "0", 0, 10000), ("b", "0", 20000, 30000)])
    ps.trace(d, 5)
    assert "Kernel time per stream" not in capsys.readouterr().out
