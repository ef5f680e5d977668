"""Host logic of bench.py that needs no GPU: the multi-GPU refusal, kernel-name parsing, and the
summaries it writes from rocprofv3 CSV files (checked on small synthetic files)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


@pytest.mark.parametrize("name,short", [
    ("void icl::(anonymous namespace)::conv2d_pers<icl::F32, 7, 8, 2>(void const*, unsigned long, void*)",
     "conv2d_pers<F32, 7, 8, 2>"),
    ("void icl::(anonymous namespace)::sep_batched_col_k<icl::BF16, 1, 64>(icl::DevImage const*, "
     "icl::ColItem const*, icl::(anonymous namespace)::ColRanges)", "sep_batched_col_k<BF16, 1, 64>"),
    ("__amd_rocclr_copyBuffer", "__amd_rocclr_copyBuffer"),
])
def test_short_kernel_names(name, short):
    assert bench._short_kernel(name) == short


@pytest.mark.parametrize("name,want", [
    ("void icl::(anonymous namespace)::conv2d_pers<icl::F32, 5, 8, 2>(...)", ("2d", 5, "pers_p8x2")),
    ("void icl::(anonymous namespace)::conv2d_lds<icl::F32, 3, 4, 2, 1>(...)", ("2d", 3, "lds_p4x2_o1")),
    ("void icl::(anonymous namespace)::sep_fused<icl::F32, 7, 32, 1>(...)", ("sep", 7, "fused_t32_c1")),
    ("void icl::(anonymous namespace)::sep_pers<icl::F32, 2, 16, 2>(...)", ("sep", 2, "pers_t16_c2")),
    ("void icl::(anonymous namespace)::sep_fused_img<icl::F32, 5, 32, 1, true>(...)",
     ("sep", 5, "fused_img4_t32_c1")),
    ("void icl::(anonymous namespace)::sep_fused_img<icl::F32, 5, 16, 2, false>(...)",
     ("sep", 5, "fused_img_t16_c2")),
    ("void icl::(anonymous namespace)::sep_colwalk<icl::F32, 3, 128>(...)", ("sep", 3, "colwalk_s128")),
    ("void icl::(anonymous namespace)::sep_fused<icl::F16, 7, 32, 1>(...)", None),
])
def test_kernel_variant_names(name, want):
    assert bench.kernel_variant(name) == want


def _write_csv(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_trace_summary_takes_the_first_run_of_exactly_the_timed_steps(tmp_path):
    """Dispatch order: the tuner's block (43 launches), the warmup (interleaved), the timed
    block (steps launches back to back), then a later workload timing the same kernel again.
    Only the timed block may feed the 'timed dispatches' column."""
    steps = 3
    k2d = "void icl::(anonymous namespace)::conv2d_pers<icl::F32, 7, 8, 2>(void const*)"
    ksep = "void icl::(anonymous namespace)::sep_fused<icl::F32, 7, 32, 1>(void const*)"
    copy = ("__amd_rocclr_copyBuffer", 5.0)
    seq = [(k2d, 50.0)] * 43 + [(ksep, 40.0), (k2d, 60.0)] + [(ksep, 41.0)] * steps + [(k2d, 100.0)] * steps \
        + [copy] + [(k2d, 70.0)] * steps + [copy]
    rows, t = [], 1000
    for i, (k, us) in enumerate(seq):
        rows.append(["KERNEL_DISPATCH", "Agent 1", 1, 0, 1, i + 1, 7, k, i + 1, t, t + int(us * 1000)])
        t += int(us * 1000) + 500
    tdir = tmp_path / "kt"
    tdir.mkdir()
    _write_csv(tdir / "kt_kernel_trace.csv", ["Kind", "Agent_Id", "Queue_Id", "Stream_Id", "Thread_Id",
                                              "Dispatch_Id", "Kernel_Id", "Kernel_Name", "Correlation_Id",
                                              "Start_Timestamp", "End_Timestamp"], rows)
    _write_csv(tdir / "kt_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs",
                                              "MaxNs", "StdDev"],
               [[k2d, 52, 1, 55000.0, 50, 50000, 100000, 1], [ksep, 4, 1, 40750.0, 50, 40000, 41000, 1]])
    line = {"value": 1.0, "unit": "Gpixel/s", "ms_per_step": 0.1, "steps": steps, "warmup": 1,
            "per_call": [{"call": "sep7", "variant": "fused_t32_c1", "us": 41.5},
                         {"call": "2d7", "variant": "pers_p8x2", "us": 100.4}],
            "roofline": {"kernel": "2d7:pers_p8x2", "launch_us": 100.4}, "extras": {}}
    bj = tmp_path / "b.json"
    bj.write_text("[bench] tuned\n" + json.dumps(line) + "\n")
    bench.write_trace_summary(str(tdir), str(bj), out_dir=str(tmp_path))
    md = (tmp_path / "kernel_trace_sweep_4096_f32.md").read_text()
    row2d = next(ln for ln in md.splitlines() if ln.startswith("| 2d7 |"))
    cells = [c.strip() for c in row2d.split("|")]
    assert cells[4] == "100.00"                          # the timed block, not the tuner's or the later one
    assert cells[8] == str(43 + 1 + 2 * steps)           # every dispatch of the kernel
    rowsep = next(ln for ln in md.splitlines() if ln.startswith("| sep7 |"))
    assert [c.strip() for c in rowsep.split("|")][4] == "41.00"
    assert "100.00 us per timed dispatch" in md
    wl = (tmp_path / "kernel_trace_workloads.md").read_text()
    assert "`conv2d_pers<F32, 7, 8, 2>` | 52 | 55.00 | 50.00 | 100.00 |" in wl
    assert "`__amd_rocclr_copyBuffer`" not in wl          # listed only if the stats file holds it


def test_counter_summary_ratios(tmp_path):
    """The ratios are plain quotients of the per-dispatch counter means (2.4 GHz, 1024 SIMDs)."""
    k = "void icl::(anonymous namespace)::conv2d_pers<icl::F32, 7, 8, 2>(void const*)"
    us = 100.0
    cyc = 1024 * us * 2.4e3
    vals = {"SQ_INSTS_VALU": cyc / 4 * 0.9, "SQ_INSTS_MFMA": 0.0, "SQ_VALU_MFMA_BUSY_CYCLES": 0.0,
            "SQ_INSTS_LDS": cyc / 4 * 0.9 * 0.05, "SQ_ACTIVE_INST_LDS": 1000.0, "SQ_LDS_BANK_CONFLICT": 2000.0,
            "SQ_WAIT_INST_LDS": 30.0, "SQ_WAIT_INST_ANY": 250.0, "SQ_WAVE_CYCLES": 1000.0}
    d = tmp_path / "sqA_sweep"
    d.mkdir()
    rows = [[k, n, v, 0, int(us * 1000)] for n, v in vals.items()]
    _write_csv(d / "sq_counter_collection.csv", ["Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp",
                                                 "End_Timestamp"], rows)
    bench.write_counter_summary([str(d)], out_dir=str(tmp_path))
    md = (tmp_path / "sq_counters.md").read_text()
    row = next(ln for ln in md.splitlines() if ln.startswith("| `conv2d_pers<F32, 7, 8, 2>`"))
    cells = [c.strip() for c in row.split("|")]
    assert cells[2] == "100.0"
    assert cells[4] == "0.90"     # vector issue share
    assert cells[6] == "0.00"     # matrix pipe idle
    assert cells[8] == "0.05"     # LDS instructions per vector instruction
    assert cells[9] == "2.00"     # conflict cycles per LDS cycle
    assert cells[10] == "0.03" and cells[11] == "0.25"


def test_calibration_factors_use_the_1gib_copies(tmp_path):
    """Counter scale factors come from the copies whose WRITE_SIZE reads 1 GiB, paired in order."""
    gib_kib = 1 << 20
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    fetch = [["__amd_rocclr_copyBuffer", "FETCH_SIZE", 32768.0],          # a 64 MiB copy (not a calibration)
             ["__amd_rocclr_copyBuffer", "FETCH_SIZE", gib_kib / 2],
             ["__amd_rocclr_copyBuffer", "FETCH_SIZE", gib_kib / 2 + 8]]
    write = [["__amd_rocclr_copyBuffer", "WRITE_SIZE", 65536.0],
             ["__amd_rocclr_copyBuffer", "WRITE_SIZE", float(gib_kib)],
             ["__amd_rocclr_copyBuffer", "WRITE_SIZE", float(gib_kib)]]
    _write_csv(tmp_path / "f.csv", hdr, fetch)
    _write_csv(tmp_path / "w.csv", hdr, write)
    fcal, wcal, f, w = bench.calib_factors(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    assert f == [gib_kib / 2, gib_kib / 2 + 8] and w == [gib_kib, gib_kib]
    assert fcal == pytest.approx(gib_kib / (gib_kib / 2 + 4)) and wcal == 1.0
    _write_csv(tmp_path / "w0.csv", hdr, write[:1] * 3)
    with pytest.raises(RuntimeError):
        bench.calib_factors(str(tmp_path / "f.csv"), str(tmp_path / "w0.csv"))
