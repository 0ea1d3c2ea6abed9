"""Products split along K (pk_params.ks > 1) through the C ABI: every MFMA
program at several share counts against the oracle (float32 within 1e-5,
bfloat16 inputs within 1e-2 relative Frobenius error), small-integer inputs
bit-exact whatever order the shares' sums enter C, accumulation, shares
left without K steps, K = 0, refused share counts, and a full-size product
checked on whole rows and columns."""
import sys

import numpy as np
import pytest
import torch

import oracle.matmul as om
from paper_1801_04348_amd import pk
from tests import inputs

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 1e-2}
# the programs of up to 512 work-items (the larger ones are never split)
F32_POINTS = [(64, 64, 32, 2, 2), (128, 64, 32, 2, 2), (64, 128, 32, 2, 2), (128, 128, 32, 2, 2),
              (256, 128, 32, 4, 2), (128, 256, 32, 2, 4)]
BF16_POINTS = [(64, 64, 64, 2, 2), (128, 64, 64, 2, 2), (64, 128, 64, 2, 2), (128, 128, 64, 2, 2),
               (256, 128, 64, 4, 2), (128, 256, 64, 2, 4), (256, 128, 32, 2, 2), (128, 256, 32, 2, 2)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def table():
    return pk.pk_case_table_build(0)


def rel_fro(c, ref):
    c = np.asarray(c, dtype=np.float64)
    num = np.linalg.norm(c - ref)
    den = np.linalg.norm(ref)
    return 0.0 if num == 0 else num / den


def fits(table, dtype, pt):
    p = pk.params(family=pk.PK_FAMILY_MFMA, bm=pt[0], bn=pt[1], bk=pt[2], wm=pt[3], wn=pt[4])
    try:
        pk.pk_kernel_name(table, p, dtype)
    except pk.PkError:
        return None
    return p


def operands(dtype, M, N, K, seed, small_int=False):
    if small_int:
        A = inputs.small_int_f32((M, K), seed=seed)
        B = inputs.small_int_f32((K, N), seed=seed + 1)
    else:
        A = inputs.uniform_f32((M, K), seed=seed)
        B = inputs.uniform_f32((K, N), seed=seed + 1)
    if dtype == "bf16":
        A, B = inputs.bf16_bits(A), inputs.bf16_bits(B)
    return A, B


def run(table, p, dtype, A, B, C=None, accumulate=False):
    M, K = A.shape
    N = B.shape[1]
    if C is None:
        C = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    pk.pk_matmul(table, p, dtype, A.cuda(), B.cuda(), C, accumulate=accumulate)
    torch.cuda.synchronize()
    return C.cpu()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("shape", [(200, 150, 1000), (65, 97, 777), (300, 260, 2051)])
def test_every_program_split(table, dtype, shape):
    M, N, K = shape
    A, B = operands(dtype, M, N, K, seed=400)
    ref = om.matmul(A, B, dtype)
    Ai, Bi = operands(dtype, M, N, K, seed=402, small_int=True)
    refi = om.matmul(Ai, Bi, dtype)
    for pt in (F32_POINTS if dtype == "f32" else BF16_POINTS):
        p = fits(table, dtype, pt)
        if p is None:
            continue
        p.ks = 2
        try:
            pk.pk_kernel_name(table, p, dtype)
        except pk.PkError:
            # no split form: only the single-stage float32 programs of 512
            # work-items, whose register cap it would exceed
            v = pk.pk_case_table_lookup(table, dtype, p)[1]
            assert dtype == "f32" and 64 * pt[3] * pt[4] == 512 and v == pk.PK_MFMA_SINGLE, pt
            continue
        for ks in (2, 3, 4, 8, 16):
            p.ks = ks
            got = run(table, p, dtype, A, B)
            assert not torch.isnan(got).any(), (pt, ks)
            err = rel_fro(got.numpy(), ref)
            assert err <= TOL[dtype], (pt, ks, err)
            # small integers: every partial sum exact, so any order is exact
            assert np.array_equal(run(table, p, dtype, Ai, Bi).numpy().astype(np.float64), refi), (pt, ks)
        say("%s %s %s ok" % (dtype, shape, pk.pk_kernel_name(table, p, dtype)))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_unaligned_rows_split(table, dtype):
    # packed odd leading dimensions: the element-load twins, split
    M, N, K = 77, 45, 1203
    A, B = operands(dtype, M, N, K, seed=410)
    ref = om.matmul(A, B, dtype)
    for pt in (F32_POINTS[:4] if dtype == "f32" else BF16_POINTS[:4]):
        p = fits(table, dtype, pt)
        p.ks = 4
        assert rel_fro(run(table, p, dtype, A, B).numpy(), ref) <= TOL[dtype], pt


def test_accumulate_and_empty_shares(table):
    M, N, K = 130, 70, 40          # 2 K steps of 32: shares 3..8 of ks = 8 hold none
    A, B = operands("f32", M, N, K, seed=420)
    ref = om.matmul(A, B, "f32")
    C0 = inputs.uniform_f32((M, N), seed=422)
    p = fits(table, "f32", (64, 64, 32, 2, 2))
    p.ks = 8
    got = run(table, p, "f32", A, B)
    assert rel_fro(got.numpy(), ref) <= 1e-5
    got = run(table, p, "f32", A, B, C=C0.cuda(), accumulate=True)
    assert rel_fro(got.numpy(), ref + C0.double().numpy()) <= 1e-5


def test_k0_clears_or_keeps(table):
    p = fits(table, "f32", (128, 128, 32, 2, 2))
    p.ks = 4
    A = torch.empty((50, 0), dtype=torch.float32)
    B = torch.empty((0, 60), dtype=torch.float32)
    assert np.all(run(table, p, "f32", A, B).numpy() == 0.0)
    C0 = inputs.uniform_f32((50, 60), seed=430)
    assert torch.equal(run(table, p, "f32", A, B, C=C0.cuda(), accumulate=True), C0)


def test_refused_share_counts(table):
    A, B = operands("f32", 64, 64, 256, seed=440)
    C = torch.empty((64, 64), dtype=torch.float32, device="cuda")
    p = fits(table, "f32", (64, 64, 32, 2, 2))
    p.ks = 17
    with pytest.raises(pk.PkError) as e:
        pk.pk_matmul(table, p, "f32", A.cuda(), B.cuda(), C)
    assert e.value.code == pk.PK_ERR_INVALID_ARG
    # a program of 1024 work-items (feasible on a machine whose block
    # register budget admits it) is never split
    m = pk.pk_machine_query(0)
    m.regs_block = max(m.regs_block, 131072)
    big = pk.pk_case_table_build(0, m)
    r = fits(big, "f32", (256, 256, 32, 4, 4))
    r.ks = 2
    with pytest.raises(pk.PkError) as e:
        pk.pk_matmul(big, r, "f32", A.cuda(), B.cuda(), C)
    assert e.value.code == pk.PK_ERR_INVALID_ARG
    q = pk.params(bx=16, by=16, s=1, ks=2)  # a VALU program
    with pytest.raises(pk.PkError) as e:
        pk.pk_matmul(table, q, "f32", A.cuda(), B.cuda(), C)
    assert e.value.code == pk.PK_ERR_INVALID_ARG


def test_measure_offers_splits_where_tiles_are_few(table):
    M, N, K = 512, 512, 8192
    res = pk.pk_measure(table, "f32", M, N, K)
    split = [(p, s) for p, s in res if p.ks > 1]
    assert split, "no split candidate at 512 x 512 x 8192"
    assert all(np.isfinite(s) and s > 0 for _, s in res)
    best = min(res, key=lambda r: r[1])
    say("512x512x8192: fastest %s ks=%d %.1f us; fastest unsplit %.1f us" % (
        pk.pk_kernel_name(table, best[0], "f32"), best[0].ks, best[1] * 1e6,
        min(s for p, s in res if p.ks <= 1) * 1e6))
    # no split at the sweep's largest shape: tiles enough for every unit
    assert not [p for p, _ in pk.pk_measure(table, "f32", 8192, 8192, 1024) if p.ks > 1]


def test_full_size_split_rows_and_columns(table):
    M, N, K = 1000, 1000, 8192
    A = inputs.uniform_f32((M, K), seed=450)
    B = inputs.uniform_f32((K, N), seed=451)
    p = fits(table, "f32", (128, 128, 32, 2, 2))
    p.ks = 4
    got = run(table, p, "f32", A, B)
    ku = K * 2.0 ** -24
    Aa, Ba = A.abs(), B.abs()
    for i in (0, 517, M - 1):
        ref = om.matmul(A[i:i + 1], B, "f32")[0]
        bound = ku / (1 - ku) * om.matmul(Aa[i:i + 1], Ba, "f32")[0]
        assert np.all(np.abs(got[i].double().numpy() - ref) <= bound), i
    for j in (0, 333, N - 1):
        ref = om.matmul(A, B[:, j:j + 1].contiguous(), "f32")[:, 0]
        bound = ku / (1 - ku) * om.matmul(Aa, Ba[:, j:j + 1].contiguous(), "f32")[:, 0]
        assert np.all(np.abs(got[:, j].double().numpy() - ref) <= bound), j
