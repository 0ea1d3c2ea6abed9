"""HBM traffic per launch of the benchmark's dominant kernel from rocprofv3
counters, calibrated by a copy of known size.

Two counter passes over the benchmark command, one counter each (each pass a
run of its own), with the calibration copy switched on:

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d D1 -o fetch -- \\
        python3 bench.py --steps 1 --warmup 1 --no-cpu-baseline --sweep-only --machine M.json --calibrate-copy
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d D2 -o write -- \\
        python3 bench.py --steps 1 --warmup 1 --no-cpu-baseline --sweep-only --machine M.json --calibrate-copy
    python3 paper_1801_04348_amd/traffic.py --fetch D1 --write D2 --kernel NAME --out profiles/traffic_NAME.json
    python3 paper_1801_04348_amd/traffic.py --fetch D1 --write D2 --out-dir profiles   # every kernel

The calibration copy (a float32 add of zero over 256 MiB: reads 256 MiB and
writes 256 MiB) gives, per counter, factor = known bytes / counter bytes; the
kernel's bytes per launch are its mean counter value (in KiB per dispatch)
over its launches in the timed region -- the dispatches between the fourth
and fifth copy (see profwindow.py), the launches the benchmark's `achieved`
averages over -- times that factor.  The result records a hash of the
kernel sources so the benchmark ignores it once the kernels change.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)
import profwindow  # noqa: E402
COPY_BYTES = 256 << 20
KERNEL_SOURCES = ("csrc/kernels/mfma.hpp", "csrc/kernels/valu.hpp", "csrc/kernels/kargs.hpp")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_per_dispatch(d, counter):
    """[(dispatch id, kernel name, counter value summed over instances)] in
    dispatch order."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no counter_collection.csv under %s" % d)
    per = {}
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != counter:
                    continue
                key = (int(r.get("Dispatch_Id", 0)), r.get("Kernel_Name", ""))
                per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    return [(k[0], k[1], v) for k, v in sorted(per.items())]


def kernel_bytes(fetch_dir, write_dir, kernels=None):
    """{kernel: record} for each library kernel of the timed window (or only
    `kernels`): per counter the calibration, launches and KiB per launch,
    and the scaled bytes per launch."""
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = counter_per_dispatch(d, counter)
        # the marker copies: the benchmark's float32 adds (not the runtime's
        # fill kernels, which also write large buffers)
        big = lambda r: r["value"] * 1024 > COPY_BYTES / 4 and "add" in r["Kernel_Name"].lower()  # noqa: E731
        recs = [{"Dispatch_Id": i, "Kernel_Name": name, "value": v} for i, name, v in rows]
        copies = sorted(r["value"] for r in recs if not r["Kernel_Name"].startswith("pk_") and big(r))
        if not copies:
            raise SystemExit("missing calibration copies for %s" % counter)
        copy_kib = copies[len(copies) // 2]
        factor = COPY_BYTES / (copy_kib * 1024.0)
        per = {}
        for r in profwindow.timed_window(recs, big=big):
            if kernels is None or r["Kernel_Name"] in kernels:
                per.setdefault(r["Kernel_Name"], []).append(r["value"])
        for name, vals in per.items():
            out = res.setdefault(name, {"kernel": name, "source_sha256": kernel_source_hash(),
                                        "copy_bytes": COPY_BYTES, "bytes_per_launch": 0.0})
            b = sum(vals) / len(vals) * 1024.0 * factor
            out[counter] = {"copy_kib": copy_kib, "factor": factor, "launches": len(vals),
                            "kernel_kib_per_launch": sum(vals) / len(vals), "bytes_per_launch": b}
            out["bytes_per_launch"] += b
    return {k: v for k, v in res.items() if "FETCH_SIZE" in v and "WRITE_SIZE" in v}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--kernel", default=None, help="one kernel (written to --out); default every kernel")
    ap.add_argument("--out", default=None, help="output file for --kernel")
    ap.add_argument("--out-dir", default=None, help="without --kernel: one traffic_<kernel>.json per kernel here")
    args = ap.parse_args()
    if args.kernel:
        res = kernel_bytes(args.fetch, args.write, {args.kernel})
        if args.kernel not in res:
            raise SystemExit("no %s dispatches in the timed window" % args.kernel)
        with open(args.out, "w") as f:
            json.dump(res[args.kernel], f, indent=1)
        print(json.dumps(res[args.kernel]))
        return 0
    res = kernel_bytes(args.fetch, args.write)
    if args.out_dir:
        os.makedirs(args.out_dir, exist_ok=True)
        for name, rec in res.items():
            with open(os.path.join(args.out_dir, "traffic_%s.json" % name), "w") as f:
                json.dump(rec, f, indent=1)
    print(json.dumps({k: round(v["bytes_per_launch"]) for k, v in res.items()}, indent=1))
    return 0


if __name__ == "__main__":
    sys.exit(main())
