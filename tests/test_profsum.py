"""The rocprofv3 summary tool (CPU): per-kernel durations from a kernel trace and per-kernel
counter means from a counter collection."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2210_03211_amd import profsum  # noqa: E402


def test_trace_and_counter_summaries(tmp_path):
    d = tmp_path / "run" / "host"
    d.mkdir(parents=True)
    (d / "run_kernel_trace.csv").write_text(
        "Kernel_Name,Start_Timestamp,End_Timestamp\n"
        "\"k_a(Ctx, QStep)\",1000,11000\n"
        "\"k_a(Ctx, QStep)\",20000,50000\n"
        "\"void k_b<true>(int)\",60000,61000\n")
    lines = profsum.trace_summary(str(tmp_path), min_total_ms=0.0)
    assert lines[1].split() == ["k_a", "2", "0.0", "20.00", "10.00", "30.00"]
    assert lines[2].split()[0] == "k_b<true>"
    assert profsum.trace_summary(str(tmp_path), min_total_ms=1.0) == lines[:1]
    (d / "run_counter_collection.csv").write_text(
        "Kernel_Name,Counter_Name,Counter_Value\n"
        "k_a(Ctx),FETCH_SIZE,10\nk_a(Ctx),FETCH_SIZE,30\n"
        "__amd_rocclr_copyBuffer,FETCH_SIZE,4\n__amd_rocclr_copyBuffer,FETCH_SIZE,8\n")
    out = profsum.pmc_summary(str(tmp_path))
    assert out[0].split() == ["__amd_rocclr_copyBuffer", "n=2", "FETCH_SIZE=6", "FETCH_SIZE_max=8"]
    assert out[1].split() == ["k_a", "n=2", "FETCH_SIZE=20"]
    assert profsum.pmc_summary(str(tmp_path), "^k_") == out[1:]
