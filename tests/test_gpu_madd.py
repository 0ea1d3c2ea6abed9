"""Matrix-addition leaves (Section 1, Fig. 1 and Fig. 2) against the oracle,
bit for bit, through the C ABI: every leaf and every program where it fits,
on ragged shapes, in wrapping int32 and float32; large sizes sampled."""
import sys

import numpy as np
import pytest
import torch

import oracle.enumerate as en
import oracle.madd as om
from paper_1801_04348_amd import pk
from tests import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def table():
    return pk.pk_case_table_build(0)


@pytest.fixture(scope="module")
def fit(table):
    d = pk.pk_case_table_describe(table)
    inst = en.InstanceData(d["instances"])
    m = d["machine"]
    return lambda dt, v, pt: en.fits(inst, en.MADD, dt, v, pt, 0, m["regs_block"], m["max_threads_block"])


def run(table, p, dtype, A, B):
    C = torch.full(A.shape, -7, dtype=A.dtype, device="cuda")
    if A.stride(0) != A.shape[1]:            # same row layout as A: leading dimension 516
        C = torch.full((A.shape[0], A.stride(0)), -7, dtype=A.dtype, device="cuda")[:, :A.shape[1]]
    pk.pk_madd(table, p, dtype, A, B, C)
    torch.cuda.synchronize()
    return C.cpu()


@pytest.fixture(scope="module")
def ragged():
    # 517 columns: element accesses; a 514-column view of 516-wide rows:
    # 16-byte aligned rows (wide accesses) with a partial group at the end
    A = inputs.full_range_i32((333, 517), seed=11)
    B = inputs.full_range_i32((333, 517), seed=12)
    Af = inputs.uniform_f32((333, 517), seed=13)
    Bf = inputs.uniform_f32((333, 517), seed=14)
    out = [(A.cuda(), B.cuda(), om.madd(A, B, "i32")), (Af.cuda(), Bf.cuda(), om.madd(Af, Bf, "f32"))]
    Av, Bv = A[:, :516].contiguous().cuda()[:, :514], B[:, :516].contiguous().cuda()[:, :514]
    Afv, Bfv = Af[:, :516].contiguous().cuda()[:, :514], Bf[:, :516].contiguous().cuda()[:, :514]
    out += [(Av, Bv, om.madd(A[:, :514], B[:, :514], "i32")), (Afv, Bfv, om.madd(Af[:, :514], Bf[:, :514], "f32"))]
    return out


@pytest.mark.parametrize("bx", [64, 128, 256])
@pytest.mark.parametrize("by", [1, 2, 4])
def test_every_leaf_and_program(table, fit, ragged, bx, by):
    for dt, dtype, (A, B, ref) in ((1, "i32", ragged[0]), (0, "f32", ragged[1]), (1, "i32", ragged[2]),
                                   (0, "f32", ragged[3])):
        for s in (1, 2, 4, 8):
            p = pk.params(family=pk.PK_FAMILY_MADD, bx=bx, by=by, s=s)
            leaf, var = pk.pk_case_table_lookup(table, dtype, p)
            say("madd %s E=(%d,%d,%d) leaf %d variant %d" % (dtype, bx, by, s, leaf, var))
            got = run(table, pk.params(family=pk.PK_FAMILY_MADD, leaf=leaf, bx=bx, by=by, s=s), dtype, A, B)
            assert np.array_equal(got.numpy().view(np.int32), ref.view(np.int32))
            for v in (0, pk.PK_VALU_GRAN):
                q = pk.params(family=pk.PK_FAMILY_MADD, variant=v, bx=bx, by=by, s=s)
                if fit(dt, v, (bx, by, s)):
                    got = run(table, q, dtype, A, B)
                    assert np.array_equal(got.numpy().view(np.int32), ref.view(np.int32)), (bx, by, s, v)
                else:
                    with pytest.raises(pk.PkError):
                        run(table, q, dtype, A, B)


def test_tiny_empty_and_leading_dimensions(table):
    for M, N in [(1, 1), (1, 7), (9, 1), (3, 5), (65, 33), (2, 2049)]:
        A = inputs.full_range_i32((M, N), seed=M * 10 + N)
        B = inputs.full_range_i32((M, N), seed=M * 10 + N + 1)
        assert np.array_equal(run(table, None, "i32", A.cuda(), B.cuda()).numpy(), om.madd(A, B, "i32")), (M, N)
    E = torch.empty((0, 5), dtype=torch.float32, device="cuda")
    pk.pk_madd(table, None, "f32", E, E, E)
    big = inputs.uniform_f32((40, 80), seed=3)
    bigb = inputs.uniform_f32((40, 90), seed=4)
    Cbig = torch.zeros((50, 70), dtype=torch.float32, device="cuda")
    A, B, C = big.cuda()[:, 5:61], bigb.cuda()[:, 20:76], Cbig[3:43, 7:63]
    pk.pk_madd(table, None, "f32", A, B, C)
    torch.cuda.synchronize()
    ref = om.madd(big[:, 5:61].contiguous(), bigb[:, 20:76].contiguous(), "f32")
    assert np.array_equal(C.cpu().numpy(), ref)
    assert torch.count_nonzero(Cbig[:3]).item() == 0 and torch.count_nonzero(Cbig[:, :7]).item() == 0
    with pytest.raises(pk.PkError):
        pk.pk_madd(table, None, "bf16", A, B, C)


def test_special_values_follow_ieee(table):
    bits = inputs.full_range_i32((64, 96), seed=21)
    bits2 = inputs.full_range_i32((64, 96), seed=22)
    A, B = bits.view(torch.float32), bits2.view(torch.float32)   # NaN, infinities, denormals
    got = run(table, None, "f32", A.cuda(), B.cuda()).numpy()
    ref = om.madd(A, B, "f32")
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    # every other result bit for bit: denormals are kept on both sides
    assert np.array_equal(got[~nan].view(np.int32), ref[~nan].view(np.int32))


@pytest.mark.parametrize("policy", [pk.PK_POLICY_CASE, pk.PK_POLICY_EXHAUSTIVE])
def test_large_sampled(table, policy):
    M, N = 8192, 12288
    A = inputs.full_range_i32((M, N), seed=5)
    B = inputs.full_range_i32((M, N), seed=6)
    p = pk.pk_select_madd(table, "i32", M, N, policy)
    say("madd %dx%d policy %d pick" % (M, N, policy), p)
    C = torch.empty((M, N), dtype=torch.int32, device="cuda")
    pk.pk_madd(table, p, "i32", A.cuda(), B.cuda(), C)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    i = rng.integers(0, M, 20000)
    j = rng.integers(0, N, 20000)
    Cs = C[torch.as_tensor(i, device="cuda"), torch.as_tensor(j, device="cuda")].cpu().numpy()
    An, Bn = A.numpy(), B.numpy()
    want = om.madd(An[i, j][None, :], Bn[i, j][None, :], "i32")[0]
    assert np.array_equal(Cs, want)
    assert np.array_equal(C[-300:, -700:].cpu().numpy(), om.madd(A[-300:, -700:].contiguous(), B[-300:, -700:].contiguous(), "i32"))
