"""Host logic of the profile tools: the timed-region window between the
benchmark's marker copies, and the calibrated traffic per launch."""
import csv
import json
import os
import subprocess
import sys

import pytest

from paper_1801_04348_amd import profwindow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY = "void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctor_add<float> >"


def trace_rows():
    # 3 calibration copies, warm-up and selection launches, marker, timed
    # launches, marker, more launches
    names = [COPY] * 3 + ["pk_a", "pk_b", "pk_a"] + [COPY] + ["pk_a", "pk_b", "pk_a"] + [COPY] + ["pk_a"]
    rows, t = [], 0
    for i, n in enumerate(names):
        d = 100_000 if n == COPY else (1000 if n == "pk_a" else 3000) + (500 if 7 <= i <= 9 else 0)
        rows.append({"Dispatch_Id": str(i + 1), "Kernel_Name": n, "Start_Timestamp": str(t),
                     "End_Timestamp": str(t + d)})
        t += d + 10
    return rows


def test_window_is_between_fourth_and_fifth_copy():
    rows = trace_rows()
    import random
    random.Random(0).shuffle(rows)              # dispatch order, not file order, decides
    win = profwindow.timed_window(rows)
    assert [r["Dispatch_Id"] for r in win] == ["8", "9", "10"]
    with pytest.raises(SystemExit):
        profwindow.timed_window(trace_rows()[:8])


def test_window_cli_stats(tmp_path):
    p = tmp_path / "k_kernel_trace.csv"
    rows = trace_rows()
    with open(p, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)
    out = subprocess.run([sys.executable, os.path.join(ROOT, "paper_1801_04348_amd", "profwindow.py"),
                          "--trace", str(p)], capture_output=True, text=True, check=True)
    res = json.loads(out.stdout)
    by = {k["kernel"]: k for k in res["kernels"]}
    assert res["dispatches"] == 3
    assert by["pk_a"]["calls"] == 2 and by["pk_a"]["average_us"] == 1.5
    assert by["pk_b"]["calls"] == 1 and by["pk_b"]["average_us"] == 3.5


def test_traffic_scaled_by_the_copy(tmp_path):
    # FETCH reads half the copy's true bytes -> factor 2; WRITE exact -> factor 1
    copy_kib = (256 << 20) / 1024
    for counter, cdir, copy_val, kern_val in (("FETCH_SIZE", "f", copy_kib / 2, 100.0), ("WRITE_SIZE", "w", copy_kib, 40.0)):
        d = tmp_path / cdir
        d.mkdir()
        copy = "void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctor_add<float> >"
        # a runtime fill of a large buffer between the markers must not count as one
        names = ([copy] * 3 + ["pk_k", "__amd_rocclr_fillBufferAligned", "pk_k"] + [copy] + ["pk_k", "pk_k"]
                 + [copy] + ["pk_k"])
        with open(d / "x_counter_collection.csv", "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for i, n in enumerate(names):
                v = copy_val if n in (copy, "__amd_rocclr_fillBufferAligned") else (kern_val if 7 <= i <= 8 else 999.0)
                w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": n, "Counter_Name": counter, "Counter_Value": v})
    out = tmp_path / "t.json"
    subprocess.run([sys.executable, os.path.join(ROOT, "paper_1801_04348_amd", "traffic.py"), "--fetch",
                    str(tmp_path / "f"), "--write", str(tmp_path / "w"), "--kernel", "pk_k", "--out", str(out)],
                   capture_output=True, text=True, check=True)
    res = json.load(open(out))
    assert res["FETCH_SIZE"]["launches"] == 2 and res["FETCH_SIZE"]["factor"] == 2.0
    assert res["bytes_per_launch"] == 100.0 * 1024 * 2 + 40.0 * 1024


def test_traffic_every_kernel(tmp_path):
    copy_kib = (256 << 20) / 1024
    for counter, cdir in (("FETCH_SIZE", "f"), ("WRITE_SIZE", "w")):
        d = tmp_path / cdir
        d.mkdir()
        names = [COPY] * 3 + ["pk_a"] + [COPY] + ["pk_a", "pk_b", "pk_b"] + [COPY] + ["pk_a"]
        with open(d / "x_counter_collection.csv", "w", newline="") as f:
            w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for i, n in enumerate(names):
                v = copy_kib if n == COPY else {"pk_a": 10.0, "pk_b": 30.0}[n] * (1 if 5 <= i <= 7 else 50)
                w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": n, "Counter_Name": counter, "Counter_Value": v})
    outd = tmp_path / "o"
    subprocess.run([sys.executable, os.path.join(ROOT, "paper_1801_04348_amd", "traffic.py"), "--fetch",
                    str(tmp_path / "f"), "--write", str(tmp_path / "w"), "--out-dir", str(outd)],
                   capture_output=True, text=True, check=True)
    a = json.load(open(outd / "traffic_pk_a.json"))
    b = json.load(open(outd / "traffic_pk_b.json"))
    assert a["bytes_per_launch"] == 2 * 10.0 * 1024 and a["WRITE_SIZE"]["launches"] == 1
    assert b["bytes_per_launch"] == 2 * 30.0 * 1024 and b["FETCH_SIZE"]["launches"] == 2


def test_counter_means_and_ratios(tmp_path):
    from paper_1801_04348_amd import counters
    names = [COPY] * 3 + ["pk_a"] + [COPY] + ["pk_a", "pk_a"] + [COPY]
    with open(tmp_path / "y_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, n in enumerate(names):
            # two hardware instances per counter and dispatch: summed
            for inst in range(2):
                for c, v in (("SQ_VALU_MFMA_BUSY_CYCLES", 30.0 + i), ("GRBM_GUI_ACTIVE", 50.0),
                             ("SQ_LDS_BANK_CONFLICT", 5.0), ("SQ_LDS_IDX_ACTIVE", 20.0)):
                    w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": n, "Counter_Name": c, "Counter_Value": v})
    res = counters.summarize([str(tmp_path)])
    assert list(res) == ["pk_a"] and res["pk_a"]["dispatches"] == 2
    m = res["pk_a"]["mean"]
    assert m["SQ_VALU_MFMA_BUSY_CYCLES"] == 2 * (35.0 + 36.0) / 2 and m["GRBM_GUI_ACTIVE"] == 100.0
    # GRBM_GUI_ACTIVE is summed over the 8 XCDs: 100 / 8 cycles, 1024 SIMDs, 256 CUs
    assert res["pk_a"]["ratios"] == {"mfma_util": round(71.0 / (12.5 * 1024), 4),
                                     "lds_active": round(40.0 / (12.5 * 256), 4),
                                     "lds_conflict_per_active": 0.25}
    res = counters.summarize([str(tmp_path)], durations={"pk_a": 10.0})
    assert res["pk_a"]["ratios"]["clock_ghz"] == 1.25
