"""The allocation-free grouped entry point (pk_matmul_batched_noalloc) through
the C ABI, against pk_matmul_batched (the entry point it varies): the same
products computed bit for bit alike, on two calls in a row, the second with
a smaller input; the first call's outputs untouched by the second; a layout
larger than the workspace refused before any work."""
import sys

import numpy as np
import pytest
import torch

import oracle.matmul as om
from paper_1801_04348_amd import pk
from tests import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def table():
    return pk.pk_case_table_build(0)


def products(G, seed, dtype):
    """Products of sizes log-uniform on [16, 300], every other one with rows
    padded to 8 elements, the rest packed (unaligned rows)."""
    dims = inputs.group_dims(G, seed, 16, 300)
    As, Bs, host = [], [], []
    for g, (M, N, K) in enumerate(dims):
        M, N, K = int(M), int(N), int(K)
        a = inputs.uniform_f32((M, K), seed=seed * 1009 + 2 * g)
        b = inputs.uniform_f32((K, N), seed=seed * 1009 + 2 * g + 1)
        if dtype == "bf16":
            a, b = inputs.bf16_bits(a), inputs.bf16_bits(b)
        if g % 2 == 0:
            ad = torch.zeros((M, (K + 7) // 8 * 8), dtype=a.dtype, device="cuda")
            bd = torch.zeros((K, (N + 7) // 8 * 8), dtype=b.dtype, device="cuda")
            ad[:, :K] = a.cuda()
            bd[:, :N] = b.cuda()
            ad, bd = ad[:, :K], bd[:, :N]
        else:
            ad, bd = a.cuda(), b.cuda()
        As.append(ad)
        Bs.append(bd)
        host.append((a, b))
    return dims, As, Bs, host


def outputs(dims, fill=float("nan")):
    return [torch.full((int(M), int(N)), fill, dtype=torch.float32, device="cuda") for M, N, _ in dims]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_two_calls_match_the_allocating_entry_point(table, dtype):
    tol = 1e-5 if dtype == "f32" else 1e-2
    results = []
    for G, seed in ((96, 31), (17, 37)):          # the second call smaller
        dims, As, Bs, host = products(G, seed, dtype)
        C_ref, C_na = outputs(dims), outputs(dims)
        pk.pk_matmul_batched(table, dtype, As, Bs, C_ref)
        say("%s: %d products, allocation-free call" % (dtype, G))
        pk.pk_matmul_batched_noalloc(table, dtype, As, Bs, C_na)
        torch.cuda.synchronize()
        for g in range(G):
            assert torch.equal(C_na[g].cpu(), C_ref[g].cpu()), (G, g, tuple(dims[g]))
        for g in range(0, G, 5):                   # and the oracle, on a sample
            a, b = host[g]
            ref = om.matmul(a, b, dtype)
            got = C_na[g].cpu().double().numpy()
            assert np.linalg.norm(got - ref) <= tol * np.linalg.norm(ref), (G, g)
        results.append(([c.cpu().clone() for c in C_na], C_na))
    # the second call left the first call's outputs as they were
    first_host, first_dev = results[0]
    for g in range(len(first_dev)):
        assert torch.equal(first_dev[g].cpu(), first_host[g]), g


def test_given_parameters_and_empty_products(table):
    dims, As, Bs, host = products(12, 41, "f32")
    ps = [pk.params(family=pk.PK_FAMILY_MFMA, bm=(64, 128)[g % 2], bn=64, bk=32, wm=2, wn=2, variant=0)
          for g in range(len(As))]
    C_ref, C_na = outputs(dims), outputs(dims)
    pk.pk_matmul_batched(table, "f32", As, Bs, C_ref, params=ps)
    pk.pk_matmul_batched_noalloc(table, "f32", As, Bs, C_na, params=ps)
    torch.cuda.synchronize()
    for g in range(len(As)):
        assert torch.equal(C_na[g].cpu(), C_ref[g].cpu()), g
    # no live product: nothing to do
    empty = [torch.empty((0, 5), dtype=torch.float32, device="cuda")]
    pk.pk_matmul_batched_noalloc(table, "f32", empty, [torch.empty((5, 3), device="cuda")],
                                 [torch.empty((0, 3), device="cuda")])


def test_layout_above_the_workspace_is_refused(table):
    # 60000 one-element products: 60000 descriptors of 80 bytes exceed 4 MiB
    G = 60000
    buf = torch.ones((G,), dtype=torch.float32, device="cuda")
    out = torch.full((G,), -1.0, dtype=torch.float32, device="cuda")
    As = [buf[g:g + 1].view(1, 1) for g in range(G)]
    Cs = [out[g:g + 1].view(1, 1) for g in range(G)]
    with pytest.raises(pk.PkError) as e:
        pk.pk_matmul_batched_noalloc(table, "f32", As, As, Cs)
    assert e.value.code == pk.PK_ERR_INVALID_ARG and "workspace" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(out == -1.0)            # nothing ran
