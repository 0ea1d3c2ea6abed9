"""Per-kernel statistics of the benchmark's timed region from a rocprofv3
kernel trace.

With --calibrate-copy the benchmark launches a 256 MiB device copy (a
non-library kernel) three times before anything else, once right before its
timed steps and once right after them.  In dispatch order, the library
kernels between the fourth and the fifth of those copies are exactly the
timed region's launches; their mean duration is what the benchmark's own
events measure.

    rocprofv3 --kernel-trace --stats --output-format csv -d D -o sweep -- \\
        python3 bench.py --steps 3 --warmup 1 --no-cpu-baseline --sweep-only --machine M.json --calibrate-copy
    python3 paper_1801_04348_amd/profwindow.py --trace D/sweep_kernel_trace.csv
"""
from __future__ import annotations

import argparse
import csv
import json
import sys

COPY_BYTES = 256 << 20


def is_copy(name: str) -> bool:
    return not name.startswith("pk_")


def timed_window(rows, key="Dispatch_Id", name_key="Kernel_Name", big=None):
    """Rows strictly between the fourth and fifth copy dispatches, in
    dispatch order.  `big(row)` tells a calibration copy from other
    non-library kernels (by duration or counter value); default: every
    non-library kernel whose name has "add" in it."""
    rows = sorted(rows, key=lambda r: int(r[key]))
    if big is None:
        big = lambda r: "add" in r[name_key].lower()  # noqa: E731
    marks = [i for i, r in enumerate(rows) if is_copy(r[name_key]) and big(r)]
    if len(marks) < 5:
        raise SystemExit("expected at least 5 copy dispatches (run the benchmark with --calibrate-copy), found %d"
                         % len(marks))
    lo, hi = marks[3], marks[4]
    return [r for r in rows[lo + 1:hi] if r[name_key].startswith("pk_")]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True, help="rocprofv3 *_kernel_trace.csv")
    ap.add_argument("--all", action="store_true",
                    help="every library dispatch of the trace, not the timed window (runs without markers)")
    ap.add_argument("--by-grid", action="store_true",
                    help="one line per kernel and grid size (the same kernel on different problem sizes)")
    args = ap.parse_args()
    with open(args.trace) as f:
        rows = list(csv.DictReader(f))
    win = [r for r in rows if r["Kernel_Name"].startswith("pk_")] if args.all else timed_window(rows)
    stats = {}
    for r in win:
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        key = r["Kernel_Name"]
        if args.by_grid:
            key += " grid=%s" % r.get("Grid_Size_X", r.get("Grid_Size", "?"))
        s = stats.setdefault(key, [0, 0, None, 0])
        s[0] += 1
        s[1] += d
        s[2] = d if s[2] is None else min(s[2], d)
        s[3] = max(s[3], d)
    total = sum(v[1] for v in stats.values())
    out = [{"kernel": k, "calls": v[0], "total_ms": round(v[1] / 1e6, 3), "average_us": round(v[1] / v[0] / 1e3, 2),
            "share_pct": round(100.0 * v[1] / total, 2), "min_us": round(v[2] / 1e3, 2), "max_us": round(v[3] / 1e3, 2)}
           for k, v in sorted(stats.items(), key=lambda kv: -kv[1][1])]
    print(json.dumps({"dispatches": len(win), "kernels": out}, indent=1))


if __name__ == "__main__":
    sys.exit(main())
