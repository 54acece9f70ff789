"""The profiler-summary tool: kernel names shortened, the implicit-step CG
kernel split into its launch roles by dispatch order, the step window, and
byte counters scaled by the copy calibration."""
import csv
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2302_12519_amd import profsum  # noqa: E402

PCG = "void ep::(anonymous namespace)::k_pcg_step<float, true>(int, int const*)"
INIT = "void ep::(anonymous namespace)::k_be_init<float, true>(int, int const*)"
GEMV = "_ZN2ep12_GLOBAL__N_113k_coarse_gemvEiPKDF16_fPKfPfPKNS_9CGScalarsE"
COPY = "__amd_rocclr_copyBuffer"


def test_short_names():
    assert profsum.short_name(PCG) == "k_pcg_step<float, true>"
    assert profsum.short_name(INIT) == "k_be_init<float, true>"
    assert profsum.short_name(GEMV) == "k_coarse_gemv"
    assert profsum.short_name(COPY) == COPY


def _trace(path, seq):
    """seq: (name, duration ns) in dispatch order."""
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        t = 1000
        for i, (name, dur) in enumerate(seq, start=1):
            w.writerow(["KERNEL_DISPATCH", i, name, t, t + dur])
            t += dur + 500


def _rows(text):
    out = {}
    for line in text.splitlines()[1:]:
        parts = line.rsplit(None, 5)
        out[parts[0].strip()] = [float(x) for x in parts[1:]]
    return out


def test_trace_roles_and_window(tmp_path, capsys):
    # step 0: init, launch 0, two iterations, last update; step 1: init,
    # launch 0, one iteration, last update
    seq = [(INIT, 100_000), (PCG, 70_000), (PCG, 100_000), (PCG, 110_000), (PCG, 20_000),
           (INIT, 120_000), (PCG, 80_000), (PCG, 90_000), (PCG, 22_000)]
    p = tmp_path / "trace.csv"
    _trace(p, seq)
    profsum.trace(str(p))
    rows = _rows(capsys.readouterr().out)
    it = rows["k_pcg_step<float, true> (iteration)"]
    assert it[0] == 3 and it[1] == pytest.approx(100.0)
    assert rows["k_pcg_step<float, true> (launch 0)"][:2] == [2, pytest.approx(75.0)]
    assert rows["k_pcg_step<float, true> (last x update)"][:2] == [2, pytest.approx(21.0)]
    assert rows["k_be_init<float, true>"][:2] == [2, pytest.approx(110.0)]
    # the window from the second implicit step on
    profsum.trace(str(p), skip_steps=1)
    rows = _rows(capsys.readouterr().out)
    assert rows["k_pcg_step<float, true> (iteration)"][:2] == [1, pytest.approx(90.0)]
    assert rows["k_be_init<float, true>"][:2] == [1, pytest.approx(120.0)]


def test_counters_calibrated(tmp_path, capsys):
    p = tmp_path / "counters.csv"
    with open(p, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
                    "Start_Timestamp", "End_Timestamp"])
        # a 1 GiB copy that the counter reads as half its bytes, then a kernel
        w.writerow([1, COPY, "FETCH_SIZE", 524288.0, 0, 200_000])
        w.writerow([2, INIT, "FETCH_SIZE", 1000.0, 300_000, 301_000])
        w.writerow([3, INIT, "WRITE_SIZE", 7.0, 400_000, 401_000])
    profsum.counters(str(p), "FETCH_SIZE", 1 << 30)
    out = capsys.readouterr().out
    assert "factor 2.0000" in out
    line = [ln for ln in out.splitlines() if ln.startswith("k_be_init")][0]
    vals = line.split()
    # 1000 KiB x 2 = 2.048 MB, over 1 us = 2048 GB/s
    assert float(vals[-3]) == pytest.approx(2.05, abs=0.01)
    assert float(vals[-1]) == pytest.approx(2048, abs=1)
