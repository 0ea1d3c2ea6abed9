"""The 2-D micro-tile VALU family (PK_FAMILY_VALU2) through the C ABI: every
point of its domain with its case-table leaf and with each program forced,
on the parity configurations -- float32 256^3 within 1e-5 relative Frobenius
error of the float64 oracle, int32 1024^3 bit-exact -- plus full-range int32
(wrapping), ragged tails and accumulation."""
import sys

import numpy as np
import pytest
import torch

import oracle.enumerate as en
import oracle.matmul as om
from paper_1801_04348_amd import pk
from tests import inputs

pytestmark = pytest.mark.gpu

F32_TOL = 1e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def table():
    return pk.pk_case_table_build(0)


@pytest.fixture(scope="module")
def fit(table):
    """fit(dtype, variant, point): whether the program fits the bound machine,
    by the oracle's own accounting of its resources."""
    d = pk.pk_case_table_describe(table)
    inst = en.InstanceData(d["instances"])
    m = d["machine"]
    return lambda dt, v, pt: en.fits(inst, en.VALU2, dt, v, pt, m["lds_block"], m["regs_block"],
                                     m["max_threads_block"])


def forced(table, fit, dtype, v, pt, *args, **kw):
    """The forced program's result, or None where it does not fit (and the
    library refuses it)."""
    if fit(pk.DTYPES[dtype], v, pt):
        return run(table, P(pt, variant=v), dtype, *args, **kw)
    with pytest.raises(pk.PkError):
        run(table, P(pt, variant=v), dtype, *args, **kw)
    return None


@pytest.fixture(scope="module")
def points(table):
    d = pk.pk_case_table_describe(table)
    part = next(p for p in d["parts"] if p["family"] == pk.PK_FAMILY_VALU2 and p["dtype"] == 0)
    return [tuple(p) for p in part["points"]]


def rel_fro(c, ref):
    c = np.asarray(c, dtype=np.float64)
    num = np.linalg.norm(c - ref)
    return 0.0 if num == 0 else num / np.linalg.norm(ref)


def P(pt, **kw):
    return pk.params(family=pk.PK_FAMILY_VALU2, bx=pt[0], by=pt[1], s=pt[2], sy=pt[3], bk=pt[4], **kw)


def run(table, p, dtype, A, B, C0=None, accumulate=False):
    M, K = A.shape
    N = B.shape[1]
    out = torch.int32 if dtype == "i32" else torch.float32
    C = C0.clone() if C0 is not None else torch.full((M, N), -7, dtype=out)
    C = C.cuda()
    pk.pk_matmul(table, p, dtype, A.cuda(), B.cuda(), C, accumulate=accumulate)
    torch.cuda.synchronize()
    return C.cpu()


def test_domain_is_the_2d_points(points):
    assert len(points) == 80
    assert all(64 <= bx * by <= 256 and s in (2, 4) and sy in (2, 4) and bk in (16, 32)
               for bx, by, s, sy, bk in points)


def test_f32_256_every_point_and_program(table, fit, points):
    A = inputs.uniform_f32((256, 256), seed=0)
    B = inputs.uniform_f32((256, 256), seed=1)
    ref = om.matmul(A, B, "f32")
    for pt in points:
        leaf, var = pk.pk_case_table_lookup(table, "f32", P(pt))
        C = run(table, P(pt, leaf=leaf), "f32", A, B)
        assert rel_fro(C.numpy(), ref) <= F32_TOL, (pt, leaf)
        for v in en.VALU2_VARIANTS:            # each program forced where it fits
            C = forced(table, fit, "f32", v, pt, A, B)
            assert C is None or rel_fro(C.numpy(), ref) <= F32_TOL, (pt, v)
    say("f32 256^3: %d points x %d programs ok" % (len(points), len(en.VALU2_VARIANTS)))


def test_i32_1024_every_point_and_program_bit_exact(table, fit, points):
    A = inputs.small_int_i32((1024, 1024), seed=0)
    B = inputs.small_int_i32((1024, 1024), seed=1)
    ref = om.matmul(A, B, "i32")
    for pt in points:
        leaf, var = pk.pk_case_table_lookup(table, "i32", P(pt))
        assert np.array_equal(run(table, P(pt, leaf=leaf), "i32", A, B).numpy(), ref), pt
        for v in en.VALU2_VARIANTS:
            C = forced(table, fit, "i32", v, pt, A, B)
            assert C is None or np.array_equal(C.numpy(), ref), (pt, v)
    say("i32 1024^3: %d points x %d programs bit-exact" % (len(points), len(en.VALU2_VARIANTS)))


@pytest.mark.parametrize("shape", [(1, 1, 1), (7, 5, 3), (97, 131, 45), (300, 260, 200), (64, 1000, 17)])
def test_tails_wrapping_and_accumulate(table, fit, points, shape):
    M, N, K = shape
    Ai = inputs.full_range_i32((M, K), seed=11)
    Bi = inputs.full_range_i32((K, N), seed=12)
    refi = om.matmul(Ai, Bi, "i32")
    Af = inputs.uniform_f32((M, K), seed=13)
    Bf = inputs.uniform_f32((K, N), seed=14)
    C0 = inputs.uniform_f32((M, N), seed=15)
    reff = om.matmul(Af, Bf, "f32") + C0.double().numpy()
    for pt in points[::3]:
        for v in en.VALU2_VARIANTS:
            C = forced(table, fit, "i32", v, pt, Ai, Bi)
            assert C is None or np.array_equal(C.numpy(), refi), (pt, v)
            C = forced(table, fit, "f32", v, pt, Af, Bf, C0=C0, accumulate=True)
            assert C is None or rel_fro(C.numpy(), reff) <= F32_TOL, (pt, v)
