"""Host-side helpers of bench.py: the kernel-source hash that ties a committed
HBM-traffic profile to the code it was measured on."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import pytest

import bench  # noqa: E402

SRC = """// header comment
__global__ void k(int *a) {   /* block
comment */
    a[threadIdx.x] = 8;   // trailing
}
"""


def test_comment_and_whitespace_edits_keep_the_hash():
    h = bench._code_hash(SRC)
    assert bench._code_hash(SRC.replace("// trailing", "// another note")) == h
    assert bench._code_hash(SRC.replace("/* block\ncomment */", "")) == h
    assert bench._code_hash(SRC.replace("    a[", "\ta[")) == h


def test_code_edits_change_the_hash():
    h = bench._code_hash(SRC)
    assert bench._code_hash(SRC.replace("= 8", "= 9")) != h
    assert bench._code_hash(SRC.replace("threadIdx.x", "threadIdx.y")) != h



def _write_csv(path, header, rows):
    import csv
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_clock_summary_from_counters(tmp_path):
    """The engine clock is the XCD-summed GUI cycles over the dispatch time;
    VALU busy counts four cycles per wave instruction on 1024 SIMDs."""
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp",
           "End_Timestamp"]
    t = 500_000   # ns
    cyc = 2.0e9 * t * 1e-9            # 2 GHz
    vi = 0.5 * 1024 * cyc / 4         # half the issue slots
    rows = [[7, "void (anonymous namespace)::k_big(int)", "GRBM_GUI_ACTIVE", 8 * cyc, 1000, 1000 + t],
            [7, "void (anonymous namespace)::k_big(int)", "SQ_INSTS_VALU", vi, 1000, 1000 + t],
            [7, "void (anonymous namespace)::k_big(int)", "SQ_ACTIVE_INST_VALU", 1.25 * vi, 1000,
             1000 + t],
            [8, "void (anonymous namespace)::k_short(int)", "GRBM_GUI_ACTIVE", 8e4, 0, 5000],
            [8, "void (anonymous namespace)::k_short(int)", "SQ_INSTS_VALU", 10, 0, 5000]]
    _write_csv(str(tmp_path / "pmc" / "pmc_counter_collection.csv"), hdr, rows)
    out = tmp_path / "clock.md"
    bench.summarize_clock(str(tmp_path / "pmc"), str(out), ["cmd"])
    text = out.read_text()
    assert "| k_big | 500.0 | 2.00 | 50.0 | 1.250 | 62.5 |" in text
    assert "k_short" not in text   # under 100 us


def test_util_summary_from_counters(tmp_path):
    """GB/s from scaled FETCH/WRITE over the trace duration; flops are 64 x the
    per-instruction flop counter."""
    _write_csv(str(tmp_path / "trace" / "t_kernel_stats.csv"), ["Name", "AverageNs"],
               [["void (anonymous namespace)::k_big(int)", 1e6]])
    kh = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    copy = "void at::native::elementwise_kernel<MulFunctor>(int)"
    _write_csv(str(tmp_path / "f" / "p_counter_collection.csv"), kh,
               [["void (anonymous namespace)::k_big(int)", "FETCH_SIZE", 1e6 / 1024],
                [copy, "FETCH_SIZE", 2 ** 20 / 2 / 1024]])
    _write_csv(str(tmp_path / "w" / "p_counter_collection.csv"), kh,
               [["void (anonymous namespace)::k_big(int)", "WRITE_SIZE", 1e6 / 1024],
                [copy, "WRITE_SIZE", 2 ** 20 / 1024]])
    _write_csv(str(tmp_path / "v" / "p_counter_collection.csv"), kh,
               [["void (anonymous namespace)::k_big(int)", "SQ_INSTS_VALU", 1.0e6],
                ["void (anonymous namespace)::k_big(int)", "SQ_WAVES", 1000],
                ["void (anonymous namespace)::k_big(int)", "SQ_INSTS_VALU_FLOPS_FP64", 1e9 / 64]])
    out = tmp_path / "u.md"
    bench.summarize_util(str(tmp_path / "trace"), str(tmp_path / "v"), str(tmp_path / "f"),
                         str(tmp_path / "w"), str(out), 2 ** 20, ["cmd"])
    row = [ln for ln in out.read_text().splitlines() if ln.startswith("| k_big")][0]
    cells = [c.strip() for c in row.strip("|").split("|")]
    # 1 MB fetched at scale 2 and 1 MB written at scale 1: 3 MB in 1 ms
    assert cells[2] == "3.0" and cells[3] == "3"
    assert cells[5] == "1000"                      # VALU instructions per wave
    assert cells[7] == "1.00"                      # 1e9 flops in 1 ms = 1 TFLOP/s
    # counters that hold the calibration copy need its size (else every figure would read 0)
    with pytest.raises(ValueError):
        bench.summarize_util(str(tmp_path / "trace"), str(tmp_path / "v"), str(tmp_path / "f"),
                             str(tmp_path / "w"), str(out), 0, ["cmd"])
