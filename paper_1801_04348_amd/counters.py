"""Per-kernel means of rocprofv3 counters over a run's timed window.

    rocprofv3 --pmc SQ_WAVES SQ_BUSY_CYCLES ... --output-format csv -d D -o run -- <command>
    python3 paper_1801_04348_amd/counters.py --dir D [--dir D2 ...] [--all]

Every *counter_collection.csv under each directory is read; a dispatch's
value of a counter is the sum over the rows rocprofv3 writes for it (one per
hardware instance).  Without --all only the library dispatches between the
fourth and fifth calibration copy are kept (profwindow.timed_window: the
commands launch those copies with --calibrate-copy or from workloads.py).
Ratios printed when their counters are present (gfx950: 8 XCDs, 256 CUs,
4 SIMDs per CU; GRBM_GUI_ACTIVE comes summed over the XCDs' graphics
engines, so GRBM_GUI_ACTIVE / 8 is the kernel's length in shader-clock
cycles -- checked against kernel-trace durations at the 2.4 GHz clock):

  mfma_util        SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 x 1024
                   SIMDs): the fraction of the matrix units' cycles spent on
                   MFMAs, at the clock the kernel ran at
  cycles_per_mfma  SQ_VALU_MFMA_BUSY_CYCLES / SQ_INSTS_MFMA (64 for
                   v_mfma_f32_32x32x2_f32, 32 for v_mfma_f32_32x32x16_bf16)
  lds_active       SQ_LDS_IDX_ACTIVE / (GRBM_GUI_ACTIVE / 8 x 256 CUs): the
                   fraction of cycles a CU's LDS spent on indexed accesses
  lds_conflict_per_active  SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE (cycles
                   lost to bank conflicts per cycle the LDS spent on
                   indexed accesses)
  lds_insts_per_mfma  SQ_INSTS_LDS / SQ_INSTS_MFMA (per-wave instruction
                   counts)
  clock_ghz        with --trace (a kernel trace of the same workload):
                   GRBM_GUI_ACTIVE / 8 over the kernel's mean duration
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)
import profwindow  # noqa: E402


def dispatches(d):
    """{dispatch id: {"Kernel_Name": name, counter: value, ...}}."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % d)
    out = {}
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                i = int(r.get("Dispatch_Id", 0))
                rec = out.setdefault(i, {"Dispatch_Id": i, "Kernel_Name": r.get("Kernel_Name", "")})
                c = r["Counter_Name"]
                rec[c] = rec.get(c, 0.0) + float(r["Counter_Value"])
    return out


XCDS, CUS, SIMDS_PER_CU = 8, 256, 4


def ratios(m, duration_ns=None):
    out = {}
    cycles = m.get("GRBM_GUI_ACTIVE", 0.0) / XCDS
    if cycles > 0:
        if "SQ_VALU_MFMA_BUSY_CYCLES" in m:
            out["mfma_util"] = round(m["SQ_VALU_MFMA_BUSY_CYCLES"] / (cycles * CUS * SIMDS_PER_CU), 4)
        if "SQ_LDS_IDX_ACTIVE" in m:
            out["lds_active"] = round(m["SQ_LDS_IDX_ACTIVE"] / (cycles * CUS), 4)
        if duration_ns:
            out["clock_ghz"] = round(cycles / duration_ns, 3)
    pairs = (("cycles_per_mfma", "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_INSTS_MFMA"),
             ("lds_conflict_per_active", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE"),
             ("lds_insts_per_mfma", "SQ_INSTS_LDS", "SQ_INSTS_MFMA"))
    for name, a, b in pairs:
        if a in m and b in m and m[b] > 0:
            out[name] = round(m[a] / m[b], 4)
    return out


def mean_durations(trace, all_dispatches=False):
    """{kernel: mean duration in ns} over a kernel trace's timed window."""
    with open(trace) as f:
        rows = list(csv.DictReader(f))
    win = [r for r in rows if r["Kernel_Name"].startswith("pk_")] if all_dispatches else profwindow.timed_window(rows)
    acc = {}
    for r in win:
        s = acc.setdefault(r["Kernel_Name"], [0, 0])
        s[0] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        s[1] += 1
    return {k: v[0] / v[1] for k, v in acc.items()}


def summarize(dirs, all_dispatches=False, durations=None):
    per = {}
    for d in dirs:
        recs = sorted(dispatches(d).values(), key=lambda r: r["Dispatch_Id"])
        if all_dispatches:
            win = [r for r in recs if r["Kernel_Name"].startswith("pk_")]
        else:
            win = profwindow.timed_window(recs)
        for r in win:
            k = per.setdefault(r["Kernel_Name"], {})
            for c, v in r.items():
                if c in ("Dispatch_Id", "Kernel_Name"):
                    continue
                s = k.setdefault(c, [0.0, 0])
                s[0] += v
                s[1] += 1
    res = {}
    for name, cs in per.items():
        means = {c: s[0] / s[1] for c, s in cs.items()}
        res[name] = {"dispatches": max(s[1] for s in cs.values()),
                     "mean": {c: round(v, 1) for c, v in sorted(means.items())},
                     "ratios": ratios(means, (durations or {}).get(name))}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dir", action="append", required=True)
    ap.add_argument("--all", action="store_true", help="every library dispatch, not the marked window")
    ap.add_argument("--trace", default=None, help="kernel trace (*_kernel_trace.csv) of the same workload: "
                                                  "adds each kernel's clock")
    args = ap.parse_args()
    durations = mean_durations(args.trace, args.all) if args.trace else None
    print(json.dumps(summarize(args.dir, args.all, durations), indent=1))


if __name__ == "__main__":
    sys.exit(main())
