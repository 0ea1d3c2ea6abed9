"""Workloads of the benchmark that profiling runs launch on their own.

Each runs a few untimed repetitions of one workload on cuda:0, bracketed by
the benchmark's calibration copies (a float32 add of zero over 256 MiB,
three times first, then once right before and once right after the
repetitions; profwindow.timed_window selects the dispatches between the last
two), so a rocprofv3 run over it reports the workload's kernels alone.
Before the window the workload runs for --warm seconds (0.25), so the
window sees the clock the workload settles at:

    python3 -m paper_1801_04348_amd.workloads grouped --dtype f32 --reps 5
    python3 -m paper_1801_04348_amd.workloads dense --dtype bf16 --n 4096 --reps 20

`grouped`: the 4096 uneven products of the grouped benchmark (M, N, K each
round(exp(U(ln 16, ln 512))) from seed 0), one plan, run eagerly `reps`
times (f32 or bf16).  `dense`: one square product of order n (f32, bf16, or
full-range i32), CASE pick (or --policy, or the MFMA program --program
names).
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COPY_BYTES = 256 << 20


def grouped_operands(torch, inputs, dtype, G=4096, seed=0):
    """The grouped benchmark's products: sizes from `inputs.group_dims`,
    operands packed in three device buffers with the rows of A and B padded
    to 8 elements (A from seed 11, B from seed 12, uniform on [-1, 1), rounded
    to bfloat16 for dtype "bf16"), C float32 packed.  Returns (dims, As, Bs,
    Cs) with per-product views."""
    import numpy as np
    dims = inputs.group_dims(G, seed=seed)
    lda = (dims[:, 2] + 7) // 8 * 8
    ldb = (dims[:, 1] + 7) // 8 * 8
    offA = np.concatenate([[0], np.cumsum(dims[:, 0] * lda)])
    offB = np.concatenate([[0], np.cumsum(dims[:, 2] * ldb)])
    offC = np.concatenate([[0], np.cumsum(dims[:, 0] * dims[:, 1])])
    Ah = inputs.uniform_f32((int(offA[-1]),), seed=11)
    Bh = inputs.uniform_f32((int(offB[-1]),), seed=12)
    if dtype == "bf16":
        Ah, Bh = inputs.bf16_bits(Ah), inputs.bf16_bits(Bh)
    Ad, Bd = Ah.cuda(), Bh.cuda()
    Cd = torch.empty((int(offC[-1]),), dtype=torch.float32, device="cuda")
    As, Bs, Cs = [], [], []
    for g, (M, N, K) in enumerate(dims):
        M, N, K = int(M), int(N), int(K)
        As.append(Ad[offA[g]:offA[g + 1]].view(M, int(lda[g]))[:, :K])
        Bs.append(Bd[offB[g]:offB[g + 1]].view(K, int(ldb[g]))[:, :N])
        Cs.append(Cd[offC[g]:offC[g + 1]].view(M, N))
    return dims, As, Bs, Cs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["grouped", "dense"])
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "i32"])
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--policy", default="case", choices=["case", "exhaustive"])
    ap.add_argument("--warm", type=float, default=0.25, help="seconds of untimed runs before the first marker")
    ap.add_argument("--program", default=None,
                    help="dense: run this MFMA program instead of the policy's pick, "
                         "as bm,bn,bk,wm,wn[,variant] (variant 1: one LDS stage)")
    args = ap.parse_args()

    import torch

    from paper_1801_04348_amd import pk
    from tests import inputs

    torch.cuda.init()
    tbl = pk.pk_case_table_build(0)
    policy = pk.PK_POLICY_CASE if args.policy == "case" else pk.PK_POLICY_EXHAUSTIVE
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)

    def marker():
        torch.add(src, 0.0, out=dst)

    for _ in range(3):
        marker()
    if args.workload == "grouped":
        dims, As, Bs, Cs = grouped_operands(torch, inputs, args.dtype)
        plan = pk.pk_grouped_plan_create(tbl, args.dtype, As, Bs, Cs, policy=policy)
        launches, tiles, chosen = plan.info()
        print("grouped %s: %d launches, %d tiles, first program %s" %
              (args.dtype, launches, tiles, pk.pk_kernel_name(tbl, chosen[0], args.dtype)), flush=True)
        plan.run()
        run = plan.run
    else:
        n = args.n
        if args.dtype == "bf16":
            A = inputs.bf16_bits(inputs.uniform_f32((n, n), seed=21)).cuda()
            B = inputs.bf16_bits(inputs.uniform_f32((n, n), seed=22)).cuda()
        elif args.dtype == "i32":
            A = inputs.full_range_i32((n, n), seed=21).cuda()
            B = inputs.full_range_i32((n, n), seed=22).cuda()
        else:
            A = inputs.uniform_f32((n, n), seed=21).cuda()
            B = inputs.uniform_f32((n, n), seed=22).cuda()
        C = torch.empty((n, n), dtype=torch.int32 if args.dtype == "i32" else torch.float32, device="cuda")
        if args.program:
            v = [int(x) for x in args.program.split(",")]
            p = pk.params(family=pk.PK_FAMILY_MFMA, bm=v[0], bn=v[1], bk=v[2], wm=v[3], wn=v[4],
                          variant=v[5] if len(v) > 5 else 0)
        else:
            p = pk.pk_select(tbl, args.dtype, n, n, n, policy)
        print("dense %s %d^3: %s" % (args.dtype, n, pk.pk_kernel_name(tbl, p, args.dtype)), flush=True)

        def run():
            pk.pk_matmul(tbl, p, args.dtype, A, B, C)
        run()
    torch.cuda.synchronize()
    # untimed runs until the clock has settled under the load
    import time
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < args.warm:
        run()
        torch.cuda.synchronize()
    marker()
    for _ in range(args.reps):
        run()
    marker()
    torch.cuda.synchronize()
    print("done: %d repetitions" % args.reps, flush=True)


if __name__ == "__main__":
    sys.exit(main())
