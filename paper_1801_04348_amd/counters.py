"""Per-kernel means of rocprofv3 counters over a run's timed window.

    rocprofv3 --pmc SQ_WAVES SQ_BUSY_CYCLES ... --output-format csv -d D -o run -- <command>
    python3 paper_1801_04348_amd/counters.py --dir D [--dir D2 ...] [--all]

Every *counter_collection.csv under each directory is read; a dispatch's
value of a counter is the sum over the rows rocprofv3 writes for it (one per
hardware instance).  Without --all only the library dispatches between the
fourth and fifth calibration copy are kept (profwindow.timed_window: the
commands launch those copies with --calibrate-copy or from workloads.py).
Ratios printed when their counters are present:

  mfma_busy_per_active   SQ_VALU_MFMA_BUSY_CYCLES / GRBM_GUI_ACTIVE
  valu_busy_per_active   SQ_ACTIVE_INST_VALU / GRBM_GUI_ACTIVE
  lds_conflict_per_active  SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE (cycles
                         lost to bank conflicts per cycle the LDS spent on
                         indexed accesses)
  lds_insts_per_mfma     SQ_INSTS_LDS / SQ_INSTS_MFMA (per-wave instruction
                         counts)

The first two are not normalised by the number of SIMDs: they are compared
between kernels of one run, and against a kernel whose flop rate is known.
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


def ratios(m):
    out = {}
    pairs = (("mfma_busy_per_active", "SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE"),
             ("valu_busy_per_active", "SQ_ACTIVE_INST_VALU", "GRBM_GUI_ACTIVE"),
             ("lds_conflict_per_active", "SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE"),
             ("lds_insts_per_mfma", "SQ_INSTS_LDS", "SQ_INSTS_MFMA"))
    for name, a, b in pairs:
        if a in m and b in m and m[b] > 0:
            out[name] = round(m[a] / m[b], 4)
    return out


def summarize(dirs, all_dispatches=False):
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
                     "mean": {c: round(v, 1) for c, v in sorted(means.items())}, "ratios": ratios(means)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dir", action="append", required=True)
    ap.add_argument("--all", action="store_true", help="every library dispatch, not the marked window")
    args = ap.parse_args()
    print(json.dumps(summarize(args.dir, args.all), indent=1))


if __name__ == "__main__":
    sys.exit(main())
