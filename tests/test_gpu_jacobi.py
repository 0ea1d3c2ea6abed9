"""1D Jacobi leaves (Section 5, Fig. 6, Table 2) against the oracle, bit for
bit, through the C ABI: every leaf and every program where it fits, on a
ragged length, several step counts, int32 over its full range (wrapping
sums) and float32; the paper's length 2^15 + 2 and a large length whole."""
import sys

import numpy as np
import pytest
import torch

import oracle.enumerate as en
import oracle.jacobi as oj
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
    return lambda dt, v, pt: en.fits(inst, en.JACOBI, dt, v, pt, m["lds_block"], m["regs_block"],
                                     m["max_threads_block"])


def run(table, p, dtype, a, steps):
    d = a.cuda()
    pk.pk_jacobi1d(table, p, dtype, d, steps)
    torch.cuda.synchronize()
    return d.cpu().numpy()


def arrays(N, seed):
    return (inputs.full_range_i32((2 * N,), seed=seed), inputs.uniform_f32((2 * N,), seed=seed + 1))


@pytest.fixture(scope="module")
def ragged():
    N = 3001
    a_i, a_f = arrays(N, 31)
    return {(dt, T): (a, oj.jacobi1d(a, T, dt)) for dt, a in (("i32", a_i), ("f32", a_f)) for T in (1, 4)}


@pytest.mark.parametrize("b", [16, 32, 64, 128, 256, 512, 1024])
def test_every_leaf_and_program(table, fit, ragged, b):
    for (dt, T), (a, ref) in ragged.items():
        dtn = 1 if dt == "i32" else 0
        for s in (1, 2, 4, 8):
            p = pk.params(family=pk.PK_FAMILY_JACOBI, bx=b, s=s)
            leaf, var = pk.pk_case_table_lookup(table, dt, p)
            say("jacobi %s T=%d E=(%d,%d) leaf %d variant %d" % (dt, T, b, s, leaf, var))
            got = run(table, pk.params(family=pk.PK_FAMILY_JACOBI, leaf=leaf, bx=b, s=s), dt, a, T)
            assert np.array_equal(got.view(np.int32), ref.view(np.int32))
            for v in VARIANTS:
                q = pk.params(family=pk.PK_FAMILY_JACOBI, variant=v, bx=b, s=s)
                if fit(dtn, v, (b, s)):
                    got = run(table, q, dt, a, T)
                    assert np.array_equal(got.view(np.int32), ref.view(np.int32)), (b, s, v)
                else:
                    with pytest.raises(pk.PkError):
                        run(table, q, dt, a, T)


def test_edges(table):
    for N in (2, 3, 4, 17, 66):
        for dt, a in zip(("i32", "f32"), arrays(N, N)):
            for T in (0, 1, 2, 3):
                ref = oj.jacobi1d(a, T, dt)
                assert np.array_equal(run(table, None, dt, a, T).view(np.int32), ref.view(np.int32)), (N, dt, T)
    with pytest.raises(pk.PkError):
        pk.pk_jacobi1d(table, None, "i32", torch.zeros(2, dtype=torch.int32, device="cuda"), 1)   # N = 1
    with pytest.raises(pk.PkError):
        pk.pk_jacobi1d(table, None, "bf16", torch.zeros(8, dtype=torch.int16, device="cuda"), 1)
    with pytest.raises(pk.PkError):
        pk.pk_jacobi1d(table, None, "i32", torch.zeros(8, dtype=torch.int32, device="cuda"), -1)
    with pytest.raises(ValueError):
        pk.pk_jacobi1d(table, None, "i32", torch.zeros(7, dtype=torch.int32, device="cuda"), 1)


@pytest.mark.parametrize("policy", [pk.PK_POLICY_CASE, pk.PK_POLICY_EXHAUSTIVE])
def test_paper_length(table, policy):
    # Table 2: four time steps over a vector of length 2^15 + 2
    N = 2 ** 15 + 2
    for dt, a in zip(("i32", "f32"), arrays(N, 41)):
        p = pk.pk_select_jacobi1d(table, dt, N, policy, steps=4)
        say("jacobi %s N=2^15+2 policy %d pick" % (dt, policy), p)
        got = run(table, p, dt, a, 4)
        assert np.array_equal(got.view(np.int32), oj.jacobi1d(a, 4, dt).view(np.int32))


def test_large_length_whole(table):
    N = 2 ** 26 + 2
    a = inputs.full_range_i32((2 * N,), seed=51)
    p = pk.pk_select_jacobi1d(table, "i32", N, steps=5)
    say("jacobi i32 N=2^26+2 pick", p)
    got = run(table, p, "i32", a, 5)
    assert np.array_equal(got, oj.jacobi1d(a, 5, "i32"))


def fused(b, s):
    return pk.params(family=pk.PK_FAMILY_JACOBI, leaf=-1, variant=pk.PK_JACOBI_FUSED, bx=b, s=s)


@pytest.mark.parametrize("b", [256, 512, 1024])
def test_several_steps_program(table, b):
    # odd step counts per launch in LDS with a recomputed halo, the last step
    # alone: both halves end as the per-step schedule leaves them, bit for bit
    # (the halves' end points differ, so a step reading the wrong half's ends
    # would show)
    for N in (3001, 2, 3, 4, 17, 300):
        for dt, a in zip(("i32", "f32"), arrays(N, N + b)):
            for s in (1, 2, 4):
                for T in (0, 1, 2, 3, 4, 5, 16, 17, 31):
                    say("jacobi fused %s N=%d B=%d s=%d T=%d" % (dt, N, b, s, T))
                    got = run(table, fused(b, s), dt, a, T)
                    assert np.array_equal(got.view(np.int32), oj.jacobi1d(a, T, dt).view(np.int32)), (N, s, T)


def test_several_steps_selection_and_refusal(table):
    N = 2 ** 20 + 2
    a = arrays(N, 61)[0]
    for policy in (pk.PK_POLICY_CASE, pk.PK_POLICY_EXHAUSTIVE):
        p = pk.pk_select_jacobi1d(table, "i32", N, policy, steps=4)
        say("jacobi N=2^20+2 4 steps policy %d pick" % policy, p, pk.pk_kernel_name(table, p, "i32"))
        assert np.array_equal(run(table, p, "i32", a, 4), oj.jacobi1d(a, 4, "i32"))
    with pytest.raises(pk.PkError):                       # no instance at this point
        run(table, fused(64, 1), "i32", a, 4)
