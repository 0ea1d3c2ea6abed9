"""Reference point on the same device: the vendor library's dense products
(torch.matmul, which ROCm serves with hipBLASLt) in bfloat16 and float32 at
orders 4096 and 8192, timed with events (three untimed calls, then 50 or 10
timed ones).  A comparison, not part of the library: nothing here runs in
the library's path.

    python3 -m paper_1801_04348_amd.vendorref
"""
from __future__ import annotations

import json
import sys


def main():
    import torch
    torch.backends.cuda.matmul.allow_tf32 = False
    torch.backends.cuda.matmul.allow_bf16_reduced_precision_reduction = False
    res = {}
    for dt, name in ((torch.bfloat16, "bf16"), (torch.float32, "f32")):
        for n in (4096, 8192):
            a = torch.rand(n, n, device="cuda", dtype=dt) - 0.5
            b = torch.rand(n, n, device="cuda", dtype=dt) - 0.5
            reps = 50 if n == 4096 else 10
            for _ in range(3):
                a @ b
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                a @ b
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            res["%s_%d" % (name, n)] = round(2 * n ** 3 / ms / 1e9, 1)
            print(name, n, "%.3f ms" % ms, "%.1f TFLOP/s" % (2 * n ** 3 / ms / 1e9), flush=True)
    print(json.dumps(res))


if __name__ == "__main__":
    sys.exit(main())
