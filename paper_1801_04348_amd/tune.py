"""Exhaustive tuner: times every feasible (leaf, E) of the case table on this
device for a list of shapes, appending to a timing store, and writes the best
choice per shape.

    python -m paper_1801_04348_amd.tune --shapes sweep  --store S.jsonl --best B.json
    python -m paper_1801_04348_amd.tune --shapes random:500:2 --store S.jsonl

Timing store (JSON lines, append-only, resumable): one record per shape
    {"machine": {...}, "dtype": "f32", "shape": [M, N, K],
     "candidates": [{"params": {...}, "name": kernel, "seconds": t}, ...]}
Operands: the leading M*K and K*N elements of two buffers from seeds 0 and
1 -- float32 uniform on [-1, 1) (as in bench.py), its bfloat16 rounding for
bf16, full-range int32 for i32.
Shape lists: "sweep" = the 216 shapes over {512, 1000, 2048, 3000, 4096,
8192}^3; "random:COUNT:SEED" = COUNT shapes log-uniform on [64, 8192]^3.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def machine_fingerprint(desc):
    m = desc["machine"]
    return {k: m[k] for k in ("arch", "cu_count", "lds_block", "regs_block", "max_threads_block", "clock_khz")}


def shape_list(spec: str):
    from tests import inputs
    if spec == "sweep":
        return [tuple(s) for s in inputs.sweep_shapes()]
    kind, count, seed = spec.split(":")
    assert kind == "random"
    return [tuple(int(x) for x in r) for r in inputs.log_uniform_shapes(int(count), int(seed))]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--shapes", default="sweep")
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--store", required=True)
    ap.add_argument("--best", default=None)
    ap.add_argument("--budget", type=float, default=1e9, help="stop after this many seconds")
    args = ap.parse_args()

    import torch

    from paper_1801_04348_amd import pk
    from tests import inputs

    tbl = pk.pk_case_table_build(0)
    desc = pk.pk_case_table_describe(tbl)
    fp = machine_fingerprint(desc)
    shapes = shape_list(args.shapes)
    done = {}
    if os.path.exists(args.store):
        with open(args.store) as f:
            for line in f:
                r = json.loads(line)
                if r["dtype"] == args.dtype and r["machine"] == fp:
                    done[tuple(r["shape"])] = r
    big = max(max(max(s[0] * s[2], s[2] * s[1]), s[0] * s[1]) for s in shapes)
    if args.dtype == "i32":
        Abuf = inputs.full_range_i32((big,), seed=0).cuda()
        Bbuf = inputs.full_range_i32((big,), seed=1).cuda()
        Cbuf = torch.empty((big,), dtype=torch.int32, device="cuda")
    else:
        Abuf = inputs.uniform_f32((big,), seed=0)
        Bbuf = inputs.uniform_f32((big,), seed=1)
        if args.dtype == "bf16":
            Abuf, Bbuf = inputs.bf16_bits(Abuf), inputs.bf16_bits(Bbuf)
        Abuf, Bbuf = Abuf.cuda(), Bbuf.cuda()
        Cbuf = torch.empty((big,), dtype=torch.float32, device="cuda")
    t_start = time.time()
    with open(args.store, "a") as out:
        for i, (M, N, K) in enumerate(shapes):
            if (M, N, K) in done:
                continue
            if time.time() - t_start > args.budget:
                print("budget reached after %d shapes" % i, flush=True)
                break
            A = Abuf[:M * K].view(M, K)
            B = Bbuf[:K * N].view(K, N)
            C = Cbuf[:M * N].view(M, N)
            t0 = time.time()
            res = pk.pk_measure(tbl, args.dtype, M, N, K, A, B, C)
            cands = [{"params": p.as_dict(), "name": pk.pk_kernel_name(tbl, p, args.dtype), "seconds": s}
                     for p, s in res]
            rec = {"machine": fp, "dtype": args.dtype, "shape": [M, N, K], "candidates": cands}
            out.write(json.dumps(rec) + "\n")
            out.flush()
            done[(M, N, K)] = rec
            b = min(cands, key=lambda c: c["seconds"])
            print("[%d/%d] %s: %d candidates in %.1fs, best %s %.1f GOP/s" % (
                i + 1, len(shapes), (M, N, K), len(cands), time.time() - t0, b["name"],
                2.0 * M * N * K / b["seconds"] / 1e9), flush=True)
    if args.best:
        best = []
        for s in shapes:
            if s in done:
                b = min(done[s]["candidates"], key=lambda c: c["seconds"])
                best.append({"shape": list(s), "params": b["params"], "name": b["name"], "seconds": b["seconds"]})
        with open(args.best, "w") as f:
            json.dump({"machine": fp, "dtype": args.dtype, "shapes": best}, f, indent=0)
        print("wrote %d best choices to %s" % (len(best), args.best), flush=True)


if __name__ == "__main__":
    main()
