"""bench.py's profile summaries (no GPU): the per-kernel mean over the last N
dispatches of a rocprofv3 kernel trace, and the source-hash gate on the
traffic figures of the committed PMC summary."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write(path, text):
    path.parent.mkdir(parents=True, exist_ok=True)
    path.write_text(text)


def test_last_dispatches_mean(tmp_path):
    # three dispatches of one kernel (the first slow), one of another
    _write(tmp_path / "x" / "run_kernel_trace.csv",
           "Kernel_Name,Start_Timestamp,End_Timestamp\n"
           "\"void gts::k::k_verify_l2<true, false, false>(a)\",100,9100\n"
           "\"void gts::k::k_verify_l2<true, false, false>(a)\",20000,20300\n"
           "\"void gts::k::k_verify_l2<true, false, false>(a)\",30000,30500\n"
           "\"void gts::k::k_bound_mfma<4>(b)\",10,30\n")
    _write(tmp_path / "x" / "run_kernel_stats.csv",
           "Name,Calls,TotalDurationNs,AverageNs,Percentage,MinNs,MaxNs\n"
           "\"void gts::k::k_verify_l2<true, false, false>(a)\",3,9800,3266,99,300,9000\n")
    text = bench.stats_summary(str(tmp_path), "t", ["cmd"], 10, last=2)
    row = [l for l in text.splitlines() if l.startswith("| `k_verify_l2") and l.count("|") == 6][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    # the last two dispatches only: (300 + 500) / 2 ns = 0.4 us
    assert cells[1] == "2" and cells[2] == "0.4" and cells[3] == "0.3" and cells[4] == "0.5"
    assert "Last 2 dispatches" in text
    # without last: only the aggregate table
    assert "Last" not in bench.stats_summary(str(tmp_path), "t", ["cmd"], 10)


def test_traffic_follows_source_hash(monkeypatch):
    e = bench._profile_entry("l2_1m_d128", "k_verify_l2")
    assert e is not None and e["bytes"] > 0
    if e["source_sha16"] == bench.source_sha16("k_verify_l2"):
        assert bench.traffic("l2_1m_d128", "k_verify_l2") == e["bytes"]
    # a changed source voids the figure
    monkeypatch.setattr(bench, "source_sha16", lambda k: "0" * 16)
    assert bench.traffic("l2_1m_d128", "k_verify_l2") is None
