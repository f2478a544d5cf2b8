"""Host logic of the benchmark (no GPU): the one-GPU contract, the algorithmic
work each roofline figure divides by, the counter summaries and the rule that a
traffic figure is only reported for the kernel sources it was measured on."""
import csv
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import synth  # noqa: E402
from paper_2112_10526_amd import rocprof_summary  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_contraction_work_per_launch():
    # 10x10 TFIM, alpha = 2: per sample N/8 bytes of spin bits, M FP32 activations and one
    # 8-byte weight, plus one pass over the P-vector in FP32
    w = synth.WORKLOADS["tfim2d_l10"]
    N, M, Ns = 100, 200, 16384
    P = N + M + N * M
    bound, work, unit, peak = bench.kernel_work("outer", w, "bf16")
    assert (bound, unit, peak) == ("hbm", "GB/s", 8.0e12)
    assert work == Ns * (N / 8 + 4 * M + 8) + 4 * P == 13524272
    bound, work, unit, _ = bench.kernel_work("qgt_w", w, "fp64")
    assert (bound, unit) == ("mfma", "TFLOP/s") and work == 2.0 * Ns * P


def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as fh:
        wr = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                            "Counter_Value"])
        wr.writeheader()
        for r in rows:
            wr.writerow(r)


def test_mfma_summary_busy_share(tmp_path, capsys):
    # one dispatch: busy cycles summed over 1024 SIMDs = half of the active cycles of
    # each (GRBM_GUI_ACTIVE arrives summed over 8 XCDs) -> 50 %
    active = 1.0e6
    rows = [dict(Dispatch_Id=1, Kernel_Name="nqs::k_gram<float>(...)", Counter_Name=c,
                 Counter_Value=v)
            for c, v in [("SQ_INSTS_VALU_MFMA_MOPS_F32", 1000.0),
                         ("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0),
                         ("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0),
                         ("SQ_VALU_MFMA_BUSY_CYCLES", 0.5 * active * 1024),
                         ("SQ_BUSY_CU_CYCLES", active * 256), ("GRBM_GUI_ACTIVE", 8 * active)]]
    _write_counters(str(tmp_path), rows)
    rocprof_summary.summarize_mfma(str(tmp_path), "cmd", "title")
    out = capsys.readouterr().out
    line = [ln for ln in out.splitlines() if "k_gram" in ln][0]
    cells = [c.strip() for c in line.strip("|").split("|")]
    assert cells[3] == "5.12e+05"  # 1000 MOPS x 512 FP32 flops
    assert cells[-1] == "50.0"


def test_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(rocprof_summary, "PROFILES", str(tmp_path))
    path = rocprof_summary.traffic_file("outer", "bf16")
    body = "- kernel_class: outer\n- hbm_bytes_per_launch: 12345\n"
    with open(path, "w") as fh:
        fh.write(body + f"- source_digest: `{rocprof_summary.source_digest('outer')}`\n")
    assert rocprof_summary.read_traffic("outer", "bf16") == 12345.0
    with open(path, "w") as fh:
        fh.write(body + "- source_digest: `0000000000000000`\n")
    assert rocprof_summary.read_traffic("outer", "bf16") is None
