"""Transposition leaves against the oracle, bit for bit, through the C ABI:
every leaf and every program where it fits, at the paper's Table 3 block
shapes and more, on ragged shapes; full size (order 2^14) sampled."""
import sys

import numpy as np
import pytest
import torch

import oracle.enumerate as en
import oracle.transpose as ot
from paper_1801_04348_amd import pk
from tests import inputs

pytestmark = pytest.mark.gpu
VARIANTS = (0, pk.PK_VALU_GRAN, pk.PK_VALU_GRAN | pk.PK_VALU_NOLDS, pk.PK_VALU_NOLDS)


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
    return lambda v, pt: en.fits(inst, en.TRANSPOSE, 0, v, pt, m["lds_block"], m["regs_block"], m["max_threads_block"])


def run(table, p, dtype, A, M, N):
    C = torch.full((N, M), -7, dtype=A.dtype, device="cuda")
    pk.pk_transpose(table, p, dtype, A, C)
    torch.cuda.synchronize()
    return C.cpu()


@pytest.fixture(scope="module")
def ragged():
    A = inputs.full_range_i32((333, 517), seed=1)
    return A.cuda(), ot.transpose(A)


@pytest.mark.parametrize("bx", [16, 32, 64])
@pytest.mark.parametrize("by", [4, 8, 16, 32])
def test_every_leaf_and_program(table, fit, ragged, bx, by):
    A, ref = ragged
    for s in (1, 2, 4, 8):
        p = pk.params(family=pk.PK_FAMILY_TRANSPOSE, bx=bx, by=by, s=s)
        try:
            leaf, var = pk.pk_case_table_lookup(table, "i32", p)
        except pk.PkError as e:
            assert e.code == pk.PK_ERR_NO_FEASIBLE_BRANCH and bx * by > 1024
            continue
        say("transpose E=(%d,%d,%d) leaf %d variant %d" % (bx, by, s, leaf, var))
        assert np.array_equal(run(table, pk.params(family=2, leaf=leaf, bx=bx, by=by, s=s), "i32", A, 333, 517).numpy(), ref)
        for v in VARIANTS:
            q = pk.params(family=2, variant=v, bx=bx, by=by, s=s)
            if fit(v, (bx, by, s)):
                assert np.array_equal(run(table, q, "i32", A, 333, 517).numpy(), ref), (bx, by, s, v)
            else:
                with pytest.raises(pk.PkError):
                    run(table, q, "i32", A, 333, 517)


def test_float_bit_patterns_and_tiny_shapes(table):
    bits = inputs.full_range_i32((64, 96), seed=2)
    f = bits.view(torch.float32)  # NaN, infinities, denormals included
    C = run(table, None, "f32", f.cuda(), 64, 96)
    assert np.array_equal(C.view(torch.int32).numpy(), ot.transpose(bits))
    for M, N in [(1, 1), (1, 7), (9, 1), (3, 5), (65, 33)]:
        A = inputs.full_range_i32((M, N), seed=M * 10 + N)
        assert np.array_equal(run(table, None, "i32", A.cuda(), M, N).numpy(), ot.transpose(A)), (M, N)


def test_leading_dimensions(table):
    big = inputs.full_range_i32((40, 80), seed=3)
    A = big.cuda()[:, 5:61]                  # 40 x 56 view, lda = 80
    Cbig = torch.zeros((70, 50), dtype=torch.int32, device="cuda")
    C = Cbig[3:59, :40]                      # 56 x 40 view, ldc = 50
    pk.pk_transpose(table, None, "i32", A, C)
    torch.cuda.synchronize()
    assert np.array_equal(C.cpu().numpy(), ot.transpose(big[:, 5:61].contiguous()))
    assert torch.count_nonzero(Cbig[:3]).item() == 0   # nothing written outside C


def test_order_2_14_sampled(table):
    n = 16384
    A = inputs.full_range_i32((n, n), seed=4)
    Ad = A.cuda()
    C = torch.empty((n, n), dtype=torch.int32, device="cuda")
    p = pk.pk_select_transpose(table, "i32", n, n)
    say("order 2^14 pick", p)
    pk.pk_transpose(table, p, "i32", Ad, C)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    i = rng.integers(0, n, 20000)
    j = rng.integers(0, n, 20000)
    Cs = C[torch.as_tensor(j, device="cuda"), torch.as_tensor(i, device="cuda")].cpu().numpy()
    sub = ot.transpose(A[:512, :256])        # a full oracle block as well
    assert np.array_equal(C[:256, :512].cpu().numpy(), sub)
    assert np.array_equal(Cs, A.numpy()[i, j])
