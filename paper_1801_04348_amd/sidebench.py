"""Side benchmarks of the paper's other examples on one GPU, each against
the HBM roofline (8 TB/s) of its compulsory traffic: matrix transposition
(Section 5.2, Table 3's order 2^14), matrix addition (Section 1), 1D Jacobi
(Section 5, Table 2's length 2^15 + 2, and 2^28 + 2) and polynomial division
(Section 5, Table 4's sizes), and the matmul programs of int32 1024^3 and
float32 256^3 against the roofline of their unit (the measured VALU ceiling;
for int32 on the matrix cores, the int8 peak over ten).  Each reports the CASE pick and the
exhaustively-best leaf.  bench.py includes them in its JSON line; alone:

    python -m paper_1801_04348_amd.sidebench      # one JSON line
"""
from __future__ import annotations

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def madd_section(tbl, pk, torch, inputs, n=16384, reps=10):
    """Matrix addition (Section 1, Fig. 1) of two order-2^14 float32 matrices:
    the CASE pick and the exhaustively-best leaf, in GB/s of compulsory
    traffic (two reads and one write per element) against 8 TB/s."""
    A = inputs.uniform_f32((n, n), seed=0).cuda()
    B = inputs.uniform_f32((n, n), seed=1).cuda()
    C = torch.empty((n, n), dtype=torch.float32, device="cuda")
    out = {"order": n, "bytes": 12 * n * n}
    for name, pol in (("case", pk.PK_POLICY_CASE), ("best", pk.PK_POLICY_EXHAUSTIVE)):
        p = pk.pk_select_madd(tbl, "f32", n, n, pol)
        pk.pk_madd(tbl, p, "f32", A, B, C)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            pk.pk_madd(tbl, p, "f32", A, B, C)
        e1.record()
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) / reps * 1e-3
        out[name] = {"kernel": pk.pk_kernel_name(tbl, p, "f32"), "gbps": round(12 * n * n / s / 1e9, 1),
                     "frac_hbm": round(12 * n * n / s / 8e12, 4)}
    return out


def jacobi_section(tbl, pk, torch, inputs, steps=4, reps=10):
    """1D Jacobi (Section 5, Fig. 6): four time steps at the paper's length
    2^15 + 2 (Table 2; launch-bound: microseconds per step) and at 2^28 + 2
    (HBM-bound), int32; CASE pick and exhaustively-best program.  `gbps` counts
    the per-step schedule's traffic (8 bytes per interior point and step);
    `frac_hbm` is the least traffic any schedule needs -- read the vector once,
    write both halves' interiors once, 12 bytes per point -- over the time,
    against 8 TB/s."""
    out = {"steps": steps}
    for label, N in (("n_2^15+2", 2 ** 15 + 2), ("n_2^28+2", 2 ** 28 + 2)):
        a = inputs.small_int_i32((2 * N,), seed=0).cuda()
        bytes_ = 8 * (N - 2) * steps
        least = 12 * (N - 2)
        row = {"bytes": bytes_, "least_bytes": least}
        for name, pol in (("case", pk.PK_POLICY_CASE), ("best", pk.PK_POLICY_EXHAUSTIVE)):
            p = pk.pk_select_jacobi1d(tbl, "i32", N, pol, steps=steps)
            pk.pk_jacobi1d(tbl, p, "i32", a, steps)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                pk.pk_jacobi1d(tbl, p, "i32", a, steps)
            e1.record()
            torch.cuda.synchronize()
            s = e0.elapsed_time(e1) / reps * 1e-3
            row[name] = {"kernel": pk.pk_kernel_name(tbl, p, "i32"), "us": round(s * 1e6, 2),
                         "gbps": round(bytes_ / s / 1e9, 1), "frac_hbm": round(least / s / 8e12, 4)}
        out[label] = row
        del a
    return out


def polydiv_section(tbl, pk, torch, reps=5):
    """Polynomial division modulo 2^31 - 1 (Section 5, Fig. 8, Table 4): a
    dividend of N = M + 100 coefficients by a monic divisor of degree M, for
    M = 2^13, 2^14, 2^15; CASE pick and exhaustively-best leaf, in
    microseconds per division and GB/s of compulsory traffic (a, b read and
    a written once per step: 12 bytes per divisor coefficient and step)."""
    P = 2147483647
    out = {"modulus": P}
    g = torch.Generator().manual_seed(0)
    for e in (13, 14, 15):
        M = 2 ** e
        N = M + 100
        a0 = torch.randint(0, P, (N,), generator=g, dtype=torch.int64).to(torch.int32).cuda()
        b = torch.randint(0, P, (M,), generator=g, dtype=torch.int64).to(torch.int32).cuda()
        a = a0.clone()
        bytes_ = 12 * M * (N - M)
        row = {"N": N, "bytes": bytes_}
        for name, pol in (("case", pk.PK_POLICY_CASE), ("best", pk.PK_POLICY_EXHAUSTIVE)):
            p = pk.pk_select_polydiv(tbl, N, M, pol)
            pk.pk_polydiv(tbl, p, a, b, P)
            ts = []
            for _ in range(reps):
                a.copy_(a0)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                pk.pk_polydiv(tbl, p, a, b, P)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e-3)
            s = sorted(ts)[len(ts) // 2]
            row[name] = {"kernel": pk.pk_kernel_name(tbl, p, "i32"), "us": round(s * 1e6, 1),
                         "gbps": round(bytes_ / s / 1e9, 1), "frac_hbm": round(bytes_ / s / 8e12, 5)}
        out["M_2^%d" % e] = row
    return out


def transpose_section(tbl, pk, torch, inputs, n=16384, reps=10):
    """Transposition of an order-2^14 float32 matrix (the paper's Table 3
    size): the CASE pick and the exhaustively-best leaf, in GB/s of compulsory
    traffic (one read and one write per element) against 8 TB/s."""
    A = inputs.uniform_f32((n, n), seed=0).cuda()
    C = torch.empty((n, n), dtype=torch.float32, device="cuda")
    out = {"order": n, "bytes": 8 * n * n}
    for name, pol in (("case", pk.PK_POLICY_CASE), ("best", pk.PK_POLICY_EXHAUSTIVE)):
        p = pk.pk_select_transpose(tbl, "f32", n, n, pol)
        pk.pk_transpose(tbl, p, "f32", A, C)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            pk.pk_transpose(tbl, p, "f32", A, C)
        e1.record()
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) / reps * 1e-3
        out[name] = {"kernel": pk.pk_kernel_name(tbl, p, "f32"), "gbps": round(8 * n * n / s / 1e9, 1),
                     "frac_hbm": round(8 * n * n / s / 8e12, 4)}
    return out


def valu_section(tbl, pk, torch, inputs, reps=20):
    """The matmul programs of int32 1024^3 (small-integer entries) and float32
    256^3: CASE pick, LEARNED pick (where the table has a model for the type),
    exhaustively-best program, and the fastest VALU program, in operations
    per second (2 M N K per product).  Each is set against the roofline of
    its unit: the measured VALU multiply-add ceiling (pk_probe_valu_rate) for
    the VALU programs; for the int32 MFMA programs the int8 matrix cores'
    5.0 POP/s over the ten int8 products each int32 one takes, 500 TOP/s."""
    mfma_i32_peak = 5.0e15 / 10
    out = {"ceiling_f32_tflops": round(pk.pk_probe_valu_rate(tbl, "f32") / 1e12, 2),
           "ceiling_i32_tops": round(pk.pk_probe_valu_rate(tbl, "i32") / 1e12, 2),
           "mfma_i32_roofline_tops": round(mfma_i32_peak / 1e12, 1)}
    for dtype, n, gen in (("i32", 1024, inputs.small_int_i32), ("f32", 256, inputs.uniform_f32)):
        A = gen((n, n), seed=0).cuda()
        B = gen((n, n), seed=1).cuda()
        C = torch.empty((n, n), dtype=A.dtype, device="cuda")
        ceiling = out["ceiling_%s_%s" % (dtype, "tops" if dtype == "i32" else "tflops")] * 1e12
        picks = []
        for name, pol in (("case", pk.PK_POLICY_CASE), ("learned", pk.PK_POLICY_LEARNED),
                          ("best", pk.PK_POLICY_EXHAUSTIVE)):
            try:
                picks.append((name, pk.pk_select(tbl, dtype, n, n, n, pol)))
            except pk.PkError as e:
                if e.code != pk.PK_ERR_COST_MODEL:  # no model for this type on the table
                    raise
        valu = [(p, t) for p, t in pk.pk_measure(tbl, dtype, n, n, n, A, B, C) if p.family != pk.PK_FAMILY_MFMA]
        picks.append(("best_valu", min(valu, key=lambda pt: pt[1])[0]))
        row = {}
        for name, p in picks:
            pk.pk_matmul(tbl, p, dtype, A, B, C)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                pk.pk_matmul(tbl, p, dtype, A, B, C)
            e1.record()
            torch.cuda.synchronize()
            s = e0.elapsed_time(e1) / reps * 1e-3
            rate = 2.0 * n ** 3 / s
            roof = mfma_i32_peak if p.family == pk.PK_FAMILY_MFMA and dtype == "i32" else ceiling
            row[name] = {"kernel": pk.pk_kernel_name(tbl, p, dtype), "us": round(s * 1e6, 1),
                         "tops": round(rate / 1e12, 2), "frac_of_roofline": round(rate / roof, 4)}
        out["%s_%d" % (dtype, n)] = row
    return out


def run_all(tbl, pk, torch, inputs):
    return {"transpose": transpose_section(tbl, pk, torch, inputs), "madd": madd_section(tbl, pk, torch, inputs),
            "jacobi": jacobi_section(tbl, pk, torch, inputs), "polydiv": polydiv_section(tbl, pk, torch),
            "valu": valu_section(tbl, pk, torch, inputs)}


def main():
    import torch

    from paper_1801_04348_amd import pk
    from tests import inputs

    torch.cuda.init()
    tbl = pk.pk_case_table_build(0)
    pk.load_shipped_models(tbl)
    print(json.dumps(run_all(tbl, pk, torch, inputs)), flush=True)


if __name__ == "__main__":
    main()
