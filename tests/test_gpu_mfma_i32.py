"""The int32 matrix-core programs (four signed base-256 digits per operand on
the int8 MFMA units) against the oracle's wrapping int32 product: bit-exact
for every point and stage count of the MFMA family's int32 part, on full-range
operands (every digit and every carry exercised), aligned rows (16-byte loads
of A) and unaligned ones (the element-load twin), edge tiles and K not a
multiple of the K tile, accumulation, and the benchmark's order 1024."""
import sys

import numpy as np
import pytest
import torch

from oracle import enumerate as en
from oracle import matmul as om
from paper_1801_04348_amd import pk
from tests import inputs

pytestmark = pytest.mark.gpu

STAGES = (0, pk.PK_MFMA_SINGLE)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def table():
    return pk.pk_case_table_build(0)


@pytest.fixture(scope="module")
def programs(table):
    """(point, stage) of every int32 MFMA program that fits the device, by the
    oracle's resource derivation; the others must be refused."""
    d = pk.pk_case_table_describe(table)
    inst = en.InstanceData(d["instances"])
    m = d["machine"]
    pts = [tuple(p) for part in d["parts"] if part["family"] == pk.PK_FAMILY_MFMA
           and part["dtype"] == pk.DTYPES["i32"] for p in part["points"]]
    assert pts
    out = []
    for pt in pts:
        for v in STAGES:
            if en.fits(inst, en.MFMA, pk.DTYPES["i32"], v, pt, m["lds_block"], m["regs_block"],
                       m["max_threads_block"]):
                out.append((pt, v))
            else:
                with pytest.raises(pk.PkError):
                    run(table, params(pt, v), torch.zeros((8, 8), dtype=torch.int32, device="cuda"),
                        torch.zeros((8, 8), dtype=torch.int32, device="cuda"))
    assert out
    return out


def params(pt, v):
    bm, bn, bk, wm, wn = pt
    return pk.params(family=pk.PK_FAMILY_MFMA, variant=v, bm=bm, bn=bn, bk=bk, wm=wm, wn=wn)


def run(table, p, A, B, C0=None, accumulate=False):
    M, N = A.shape[0], B.shape[1]
    C = C0.clone() if C0 is not None else torch.full((M, N), -123456789, dtype=torch.int32, device="cuda")
    pk.pk_matmul(table, p, "i32", A, B, C, accumulate=accumulate)
    torch.cuda.synchronize()
    return C.cpu().numpy()


def padded(X, extra, lead=0):
    """X on the device as a view into rows of len(X[0]) + extra elements,
    starting `lead` elements into each row (lead = 1: rows off alignment)."""
    R, Cn = X.shape
    Y = torch.zeros((R, Cn + extra), dtype=X.dtype)
    Y[:, lead:lead + Cn] = X
    return Y.cuda()[:, lead:lead + Cn]


@pytest.mark.parametrize("shape", [(300, 260, 200), (129, 65, 33), (64, 128, 64), (1, 1, 1), (70, 3, 0)])
def test_every_program_full_range(table, programs, shape):
    M, N, K = shape
    A = inputs.full_range_i32((M, K), seed=31 + M)
    B = inputs.full_range_i32((K, N), seed=32 + N)
    ref = om.matmul(A, B, "i32")
    Aa, Ba = padded(A, (-K) % 4), padded(B, (-N) % 4)     # rows aligned for 16-byte loads
    Au, Bu = padded(A, 2, lead=1), padded(B, 2, lead=1)   # rows one element off alignment
    for pt, v in programs:
        say("mfma i32 %s stage %d on %dx%dx%d" % (pt, v, M, N, K))
        Ca = run(table, params(pt, v), Aa, Ba)
        assert np.array_equal(Ca, ref), (pt, v, "aligned")
        Cu = run(table, params(pt, v), Au, Bu)
        assert np.array_equal(Cu, ref), (pt, v, "unaligned")


def test_accumulate_wraps(table, programs):
    M, N, K = 200, 150, 96
    A = inputs.full_range_i32((M, K), seed=41)
    B = inputs.full_range_i32((K, N), seed=42)
    C0 = inputs.full_range_i32((M, N), seed=43)
    ref = om.matmul(A, B, "i32", Cin=C0.numpy())
    for pt, v in programs:
        C = run(table, params(pt, v), A.cuda(), B.cuda(), C0=C0.cuda(), accumulate=True)
        assert np.array_equal(C, ref), (pt, v)


def test_order_1024_every_program(table, programs):
    # the side benchmark's int32 order; operands full range
    n = 1024
    A = inputs.full_range_i32((n, n), seed=21)
    B = inputs.full_range_i32((n, n), seed=22)
    ref = om.matmul(A, B, "i32")
    Ad, Bd = A.cuda(), B.cuda()
    for pt, v in programs:
        assert np.array_equal(run(table, params(pt, v), Ad, Bd), ref), (pt, v)
    # and whatever CASE picks there
    assert np.array_equal(run(table, None, Ad, Bd), ref)
