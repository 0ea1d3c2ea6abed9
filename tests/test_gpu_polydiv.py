"""Polynomial-division leaves (Section 5, Fig. 8, Table 4) against the
oracle, bit for bit, through the C ABI: every leaf and every program where
it fits on a ragged size, moduli up to 2^31 - 1, the edge cases, the paper's
sizes (M = 2^13 .. 2^15, N = M + 100) and a large divisor."""
import sys

import numpy as np
import pytest
import torch

import oracle.enumerate as en
import oracle.polydiv as opd
from paper_1801_04348_amd import pk

pytestmark = pytest.mark.gpu
VARIANTS = (0, pk.PK_VALU_GRAN, pk.PK_VALU_GRAN | pk.PK_VALU_NOLDS, pk.PK_VALU_NOLDS)
P31 = 2147483647


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def residues(n, P, seed):
    g = torch.Generator().manual_seed(seed)
    return (torch.randint(0, P, (n,), generator=g, dtype=torch.int64)).to(torch.int32)


@pytest.fixture(scope="module")
def table():
    return pk.pk_case_table_build(0)


@pytest.fixture(scope="module")
def fit(table):
    d = pk.pk_case_table_describe(table)
    inst = en.InstanceData(d["instances"])
    m = d["machine"]
    return lambda v, pt: en.fits(inst, en.POLYDIV, 1, v, pt, m["lds_block"], m["regs_block"], m["max_threads_block"])


def run(table, p, a, b, P):
    da, db = a.cuda(), b.cuda()
    pk.pk_polydiv(table, p, da, db, P)
    torch.cuda.synchronize()
    return da.cpu().numpy().view(np.uint32)


def oracle(a, b, P):
    return opd.polydiv(a.numpy().view(np.uint32), b.numpy().view(np.uint32), P)


@pytest.fixture(scope="module")
def ragged():
    M, N = 3001, 3038
    out = []
    for P, seed in ((P31, 1), (65521, 2)):
        a, b = residues(N, P, seed), residues(M, P, seed + 10)
        out.append((a, b, P, oracle(a, b, P)))
    return out


@pytest.mark.parametrize("b", [16, 32, 64, 128, 256, 512, 1024])
def test_every_leaf_and_program(table, fit, ragged, b):
    for a, bb, P, ref in ragged:
        for s in (1, 2, 4, 8):
            p = pk.params(family=pk.PK_FAMILY_POLYDIV, bx=b, s=s)
            leaf, var = pk.pk_case_table_lookup(table, "i32", p)
            say("polydiv P=%d E=(%d,%d) leaf %d variant %d" % (P, b, s, leaf, var))
            got = run(table, pk.params(family=pk.PK_FAMILY_POLYDIV, leaf=leaf, bx=b, s=s), a, bb, P)
            assert np.array_equal(got, ref)
            for v in VARIANTS:
                q = pk.params(family=pk.PK_FAMILY_POLYDIV, variant=v, bx=b, s=s)
                if fit(v, (b, s)):
                    assert np.array_equal(run(table, q, a, bb, P), ref), (b, s, v)
                else:
                    with pytest.raises(pk.PkError):
                        run(table, q, a, bb, P)


def test_edges(table):
    for N, M, P in ((0, 1, 7), (5, 5, 7), (3, 9, 7), (6, 1, 2), (40, 1, 3), (40, 39, P31), (65, 64, 65521)):
        a, b = residues(N, P, N + M), residues(M, P, N + M + 1)
        assert np.array_equal(run(table, None, a, b, P), oracle(a, b, P)), (N, M, P)
    # maximal residues: every product is (P-1)^2
    P = P31
    a = torch.full((300,), P - 1, dtype=torch.int32)
    b = torch.full((200,), P - 1, dtype=torch.int32)
    assert np.array_equal(run(table, None, a, b, P), oracle(a, b, P))
    z = torch.zeros(4, dtype=torch.int32, device="cuda")
    for P in (0, 1, 2 ** 31):
        with pytest.raises(pk.PkError):
            pk.pk_polydiv(table, None, z, z[:2], P)
    with pytest.raises(pk.PkError):
        pk.pk_polydiv(table, None, z, z[:0], 7)


@pytest.mark.parametrize("policy", [pk.PK_POLICY_CASE, pk.PK_POLICY_EXHAUSTIVE])
def test_paper_sizes(table, policy):
    for e in (13, 14, 15):
        M = 2 ** e
        N = M + 100
        a, b = residues(N, P31, e), residues(M, P31, e + 100)
        p = pk.pk_select_polydiv(table, N, M, policy)
        say("polydiv M=2^%d policy %d pick" % (e, policy), p)
        assert np.array_equal(run(table, p, a, b, P31), oracle(a, b, P31))


def test_large_divisor(table):
    M = 2 ** 22
    N = M + 40
    a, b = residues(N, P31, 77), residues(M, P31, 78)
    assert np.array_equal(run(table, None, a, b, P31), oracle(a, b, P31))


def fused(b, s):
    return pk.params(family=pk.PK_FAMILY_POLYDIV, leaf=-1, variant=pk.PK_POLYDIV_FUSED, bx=b, s=s)


@pytest.mark.parametrize("b", [64, 128, 256, 512, 1024])
def test_one_launch_program(table, ragged, b):
    # quotient recurrence then the remainder in parallel: every point, K <= 128
    for a, bb, P, ref in ragged:
        for s in (1, 2, 4, 8):
            say("polydiv fused P=%d B=%d s=%d K=%d" % (P, b, s, a.numel() - bb.numel()))
            assert np.array_equal(run(table, fused(b, s), a, bb, P), ref), (b, s)


@pytest.mark.parametrize("N,M", [(3001 + 700, 3001), (1024 + 2000, 2000), (300, 5), (1030, 6), (129, 1), (5000, 4999)])
def test_one_launch_quotient_lengths(table, N, M):
    # K = N - M across the register-slot boundary (128) up to 1024, and K > M
    a, b = residues(N, P31, N), residues(M, P31, N + 1)
    ref = oracle(a, b, P31)
    for bx, s in ((64, 1), (256, 4), (1024, 2)):
        say("polydiv fused N=%d M=%d B=%d s=%d" % (N, M, bx, s))
        assert np.array_equal(run(table, fused(bx, s), a, b, P31), ref), (bx, s)


def test_one_launch_refusals(table):
    a, b = residues(3000, 7, 1), residues(1000, 7, 2)   # K = 2000 > 1024
    with pytest.raises(pk.PkError):
        run(table, fused(256, 1), a, b, 7)
    a, b = residues(300, 7, 1), residues(200, 7, 2)
    with pytest.raises(pk.PkError):                      # workgroups of less than a wavefront
        run(table, fused(32, 1), a, b, 7)
    p = pk.pk_select_polydiv(table, 2 ** 15 + 100, 2 ** 15)
    say("polydiv M=2^15 case pick", p, pk.pk_kernel_name(table, p, "i32"))
