"""Training and evaluation of the learned cost model from timing stores.

    python -m paper_1801_04348_amd.costmodel train --store S1.jsonl [--store S2.jsonl] --out MODEL.txt
    python -m paper_1801_04348_amd.costmodel eval --model MODEL.txt --store HELDOUT.jsonl [--json OUT.json]

train: one row per (shape, candidate) of the stores (written by tune.py on
this device): the library's features of the candidate (pk_features) and its
measured seconds; rows within --near (1.3) times their shape's fastest
candidate are repeated --copies (8) times in all, so the squared error
weighs most where the choice is made (a plain mean over every candidate is
dominated by programs that never win); the network is trained on the device
by the library (pk_costmodel_train) and saved with its standardisation, the
machine and the element type it was trained on (one model per type; the
stores must not mix types).

eval: for every shape of a held-out store, the LEARNED choice as pk_select
makes it -- the candidate with the least predicted time, except that when the
best two predictions are within 5 % every candidate predicted within 5 % of
the best is measured and the fastest kept; the measurement used is the
store's own -- and the CASE choice, each scored by its measured time against
the best measured candidate:  ratio = t_best / t_pick = GF_pick / GF_best.
The CASE choice is the candidate with the least pk_estimate among those the
store holds (the ones feasible for the operands' alignment).  Reports the
geometric mean, median, 10th percentile and worst ratio, the same for the
model's own pick without measurement, the fallback rate, and the
prediction latency per shape (one launch over the shape's candidates).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MARGIN = 0.05


def load_store(paths, fingerprint):
    recs = []
    for p in paths:
        with open(p) as f:
            for line in f:
                r = json.loads(line)
                if r["machine"] == fingerprint:
                    recs.append(r)
    return recs


def fingerprint_of(pk, tbl):
    m = pk.pk_case_table_describe(tbl)["machine"]
    return {k: m[k] for k in ("arch", "cu_count", "lds_block", "regs_block", "max_threads_block", "clock_khz")}


def feature_rows(pk, tbl, rec):
    import numpy as np
    M, N, K = rec["shape"]
    # the tuner's operands are packed prefixes of 16-byte aligned buffers
    wide = pk.packed_rows_wide(rec["dtype"], N, K)
    X = np.stack([pk.pk_features(tbl, pk.params(**c["params"]), rec["dtype"], M, N, K, wide)
                  for c in rec["candidates"]])
    t = np.array([c["seconds"] for c in rec["candidates"]], dtype=np.float64)
    return X, t


def stats(ratios):
    import numpy as np
    r = np.sort(np.asarray(ratios))
    return {"shapes": int(r.size), "geomean": float(np.exp(np.mean(np.log(r)))), "median": float(np.median(r)),
            "p10": float(np.percentile(r, 10)), "worst": float(r[0])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "eval"])
    ap.add_argument("--store", action="append", required=True)
    ap.add_argument("--out", default=None)
    ap.add_argument("--model", default=None)
    ap.add_argument("--epochs", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--json", default=None)
    ap.add_argument("--near", type=float, default=1.3,
                    help="train: rows within this factor of their shape's fastest candidate are repeated")
    ap.add_argument("--copies", type=int, default=8, help="train: copies of each such row (1: no repetition)")
    args = ap.parse_args()

    import numpy as np
    import torch  # noqa: F401  (one HIP runtime: torch's, see pk.py)

    from paper_1801_04348_amd import pk

    tbl = pk.pk_case_table_build(0)
    fp = fingerprint_of(pk, tbl)
    recs = load_store(args.store, fp)
    if not recs:
        sys.exit("no timing records for this machine in %s" % args.store)

    dtypes = {r["dtype"] for r in recs}
    if len(dtypes) != 1:
        sys.exit("the stores mix element types %s: one model per type" % sorted(dtypes))
    dtype = dtypes.pop()

    if args.cmd == "train":
        Xs, ts = zip(*(feature_rows(pk, tbl, r) for r in recs))
        near = [np.repeat(np.arange(len(t_)), np.where(t_ <= args.near * t_.min(), args.copies, 1)) for t_ in ts]
        X = np.concatenate([x[i] for x, i in zip(Xs, near)]).astype(np.float32)
        t = np.concatenate([t_[i] for t_, i in zip(ts, near)])
        import time
        t0 = time.perf_counter()
        cm, loss = pk.pk_costmodel_train(tbl, X, t, epochs=args.epochs, lr=args.lr, seed=args.seed)
        train_s = time.perf_counter() - t0
        cm.set_dtype(dtype)
        pred = cm.predict(X)
        rmse = float(np.sqrt(np.mean((pred - np.log(t)) ** 2)))
        cm.save(args.out)
        print(json.dumps({"dtype": dtype, "rows": int(X.shape[0]), "distinct_rows": int(sum(len(t_) for t_ in ts)),
                          "near": args.near, "copies": args.copies, "shapes": len(recs), "epochs": args.epochs,
                          "lr": args.lr,
                          "loss_standardised": loss, "rmse_ln_seconds": rmse, "train_seconds": round(train_s, 3),
                          "ms_per_epoch": round(train_s / args.epochs * 1e3, 4), "model": args.out}), flush=True)
        return

    cm = pk.pk_costmodel_load(args.model)
    if cm.dtype() != dtype:
        sys.exit("the model was trained on %s timings, the store holds %s" % (cm.dtype(), dtype))
    pk.pk_case_table_set_costmodel(tbl, cm)
    import time
    learned, model_only, case, fallbacks, measured, infer = [], [], [], 0, 0, []
    for r in recs:
        M, N, K = r["shape"]
        X, t = feature_rows(pk, tbl, r)
        t0 = time.perf_counter()
        pred = cm.predict(X)
        infer.append(time.perf_counter() - t0)
        order = np.argsort(pred, kind="stable")
        pick = int(order[0])
        best = float(t.min())
        model_only.append(best / t[pick])
        if len(order) > 1 and math.exp(pred[order[1]] - pred[order[0]]) < 1.0 + MARGIN:
            close = [int(i) for i in order if math.exp(pred[i] - pred[order[0]]) <= 1.0 + MARGIN]
            pick = min(close, key=lambda i: t[i])
            fallbacks += 1
            measured += len(close)
        learned.append(best / t[pick])
        # CASE among the candidates the store holds (those feasible for the
        # operands' alignment), as pk_matmul's own CASE choice would be
        wide = pk.packed_rows_wide(r["dtype"], N, K)
        est = [pk.pk_estimate(tbl, pk.params(**c["params"]), r["dtype"], M, N, K, wide) for c in r["candidates"]]
        case.append(best / t[int(np.argmin(est))])
    out = {"dtype": dtype, "learned": stats(learned), "learned_without_measurement": stats(model_only), "case": stats(case),
           "fallback_rate": fallbacks / len(recs), "candidates_measured_per_fallback": measured / max(fallbacks, 1),
           "margin": MARGIN, "predict_ms_per_shape": round(1e3 * sum(infer) / len(infer), 4), "model": args.model}
    out["learned_over_case_geomean"] = out["learned"]["geomean"] / out["case"]["geomean"]
    print(json.dumps(out), flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
