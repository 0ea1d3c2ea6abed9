"""Grouped persistent launches (many independent products) through the C ABI:
each product against the oracle, bit-exact against the single-product launch
of the same program, graph replays, sentinels, and the 4096-product size."""
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


def rel_fro(c, ref):
    c = np.asarray(c, dtype=np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(c - ref)
    return 0.0 if num == 0 else num / den


def make_groups(G, seed, dtype, aligned_every=1, lo=16, hi=512):
    """Products with sizes round(exp(U(ln lo, ln hi))); every `aligned_every`-th
    product gets leading dimensions padded to 8 elements (16-byte rows), the
    others are packed tightly (rows generally unaligned)."""
    dims = inputs.group_dims(G, seed, lo, hi)
    host, dev = [], []
    for g, (M, N, K) in enumerate(dims):
        M, N, K = int(M), int(N), int(K)
        a32 = inputs.uniform_f32((M, K), seed=seed * 100003 + 2 * g)
        b32 = inputs.uniform_f32((K, N), seed=seed * 100003 + 2 * g + 1)
        a = inputs.bf16_bits(a32) if dtype == "bf16" else a32
        b = inputs.bf16_bits(b32) if dtype == "bf16" else b32
        pad = (g % aligned_every == 0)
        if pad:
            Kp, Np = (K + 7) // 8 * 8, (N + 7) // 8 * 8
            ad = torch.zeros((M, Kp), dtype=a.dtype, device="cuda")
            bd = torch.zeros((K, Np), dtype=b.dtype, device="cuda")
            ad[:, :K] = a.cuda()
            bd[:, :N] = b.cuda()
            ad, bd = ad[:, :K], bd[:, :N]
        else:
            ad, bd = a.cuda(), b.cuda()
        host.append((a, b))
        dev.append((ad, bd, torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")))
    return dims, host, dev


def row_forms(dtype, dev):
    """The grouped kernel forms a plan over these operands needs: wide (rows
    aligned for 16-byte loads: 16-byte aligned bases, leading dimensions
    multiples of 4 float32 / 8 bfloat16 elements) and element loads; each
    form runs as a launch of its own."""
    vec = 8 if dtype == "bf16" else 4
    forms = set()
    for a, b, c in dev:
        if a.shape[0] * b.shape[1] == 0:
            continue
        wide = a.shape[1] > 0 and all(t.data_ptr() % 16 == 0 and t.stride(0) % vec == 0 for t in (a, b))
        forms.add(wide)
    return forms


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_grouped_matches_oracle_and_single_launch(table, dtype):
    dims, host, dev = make_groups(96, seed=3, dtype=dtype, aligned_every=2, hi=300)
    As, Bs, Cs = zip(*dev)
    plan = pk.pk_grouped_plan_create(table, dtype, As, Bs, Cs)
    n_launch, tiles, chosen = plan.info()
    say("%s plan: %d launches, %d tiles" % (dtype, n_launch, tiles))
    plan.run()
    torch.cuda.synchronize()
    tol = 1e-5 if dtype == "f32" else 1e-2
    for g, ((a, b), (ad, bd, cd)) in enumerate(zip(host, dev)):
        ref = om.matmul(a, b, dtype)
        got = cd.cpu()
        assert not torch.isnan(got).any(), g
        assert rel_fro(got.numpy(), ref) <= tol, (g, dims[g])
        if g % 2 == 0:  # aligned: the single-product launch of the same program is bit-identical
            C1 = torch.empty_like(cd)
            pk.pk_matmul(table, chosen[g], dtype, ad, bd, C1)
            torch.cuda.synchronize()
            assert torch.equal(C1.cpu(), got), (g, dims[g], chosen[g])


def test_grouped_graph_replays_match_eager(table):
    dims, host, dev = make_groups(128, seed=5, dtype="f32", aligned_every=3)
    As, Bs, Cs = zip(*dev)
    plan = pk.pk_grouped_plan_create(table, "f32", As, Bs, Cs)
    plan.run()
    torch.cuda.synchronize()
    eager = [c.cpu().clone() for c in Cs]
    plan.capture()
    for rep in range(3):
        for c in Cs:
            c.zero_()                      # eager work between replays
        torch.cuda.synchronize()
        plan.replay()
        torch.cuda.synchronize()
        for g, c in enumerate(Cs):
            assert torch.equal(c.cpu(), eager[g]), (rep, g)


def test_batched_one_shot_and_accumulate(table):
    dims, host, dev = make_groups(40, seed=7, dtype="f32", aligned_every=1, hi=200)
    As, Bs, Cs = zip(*dev)
    pk.pk_matmul_batched(table, "f32", As, Bs, Cs)
    first = [c.cpu().clone() for c in Cs]
    for c in Cs:
        c.zero_()
    plan = pk.pk_grouped_plan_create(table, "f32", As, Bs, Cs, accumulate=True)
    plan.run()
    plan.run()
    torch.cuda.synchronize()
    for g, c in enumerate(Cs):
        assert not torch.isnan(first[g]).any()
        # small operands: every tile visited exactly once per run
        assert torch.allclose(c.cpu(), 2 * first[g], rtol=1e-6, atol=1e-6), g


def test_given_per_group_params(table):
    dims, host, dev = make_groups(12, seed=9, dtype="f32", aligned_every=1, hi=260)
    As, Bs, Cs = zip(*dev)
    p = pk.params(family=pk.PK_FAMILY_MFMA, bm=64, bn=64, bk=32, wm=2, wn=2)
    plan = pk.pk_grouped_plan_create(table, "f32", As, Bs, Cs, params=[p] * len(As))
    n_launch, tiles, chosen = plan.info()
    assert n_launch == 1
    plan.run()
    torch.cuda.synchronize()
    for (a, b), (ad, bd, cd) in zip(host, dev):
        assert rel_fro(cd.cpu().numpy(), om.matmul(a, b, "f32")) <= 1e-5


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_exhaustive_plan_picks_a_fitting_program(table, dtype):
    dims, host, dev = make_groups(64, seed=13, dtype=dtype, aligned_every=2, hi=300)
    As, Bs, Cs = zip(*dev)
    plan = pk.pk_grouped_plan_create(table, dtype, As, Bs, Cs, policy=pk.PK_POLICY_EXHAUSTIVE)
    n_launch, tiles, chosen = plan.info()
    assert n_launch == len(row_forms(dtype, dev))  # one launch per row form
    names = {pk.pk_kernel_name(table, c, dtype) for c in chosen}
    say("%s exhaustive grouped pick: %s running %s" % (dtype, plan.kernels(), sorted(names)))
    if len(names) > 1:
        assert all(k.startswith("pk_grouped_mixed_%s" % dtype) for k in plan.kernels())
    for c in Cs:
        c.fill_(float("nan"))              # the selection runs wrote C; start again
    plan.run()
    torch.cuda.synchronize()
    tol = 1e-5 if dtype == "f32" else 1e-2
    for g, ((a, b), (ad, bd, cd)) in enumerate(zip(host, dev)):
        assert rel_fro(cd.cpu().numpy(), om.matmul(a, b, dtype)) <= tol, (g, dims[g])
    with pytest.raises(pk.PkError) as e:
        pk.pk_grouped_plan_create(table, dtype, As, Bs, Cs, policy=pk.PK_POLICY_EXHAUSTIVE, accumulate=True)
    assert e.value.code == pk.PK_ERR_INVALID_ARG


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_4096_products_sampled(table, dtype):
    G = 4096
    dims = inputs.group_dims(G, seed=0)
    say("4096 products, %s: sum 2MNK = %.1f GFLOP" % (dtype, 2 * np.prod(dims, axis=1).sum() / 1e9))
    # operands packed in three large buffers with 8-element-aligned rows
    lda = (dims[:, 2] + 7) // 8 * 8
    ldb = (dims[:, 1] + 7) // 8 * 8
    offA = np.concatenate([[0], np.cumsum(dims[:, 0] * lda)])
    offB = np.concatenate([[0], np.cumsum(dims[:, 2] * ldb)])
    offC = np.concatenate([[0], np.cumsum(dims[:, 0] * dims[:, 1])])
    Ah = inputs.uniform_f32((int(offA[-1]),), seed=11)
    Bh = inputs.uniform_f32((int(offB[-1]),), seed=12)
    if dtype == "bf16":
        Ah, Bh = inputs.bf16_bits(Ah), inputs.bf16_bits(Bh)
    Ad, Bd = Ah.cuda(), Bh.cuda()
    Cd = torch.full((int(offC[-1]),), float("nan"), dtype=torch.float32, device="cuda")
    As, Bs, Cs = [], [], []
    for g, (M, N, K) in enumerate(dims):
        M, N, K = int(M), int(N), int(K)
        As.append(Ad[offA[g]:offA[g + 1]].view(M, int(lda[g]))[:, :K])
        Bs.append(Bd[offB[g]:offB[g + 1]].view(K, int(ldb[g]))[:, :N])
        Cs.append(Cd[offC[g]:offC[g + 1]].view(M, N))
    plan = pk.pk_grouped_plan_create(table, dtype, As, Bs, Cs)
    plan.capture()
    plan.replay()
    torch.cuda.synchronize()
    assert not torch.isnan(Cd).any()
    rng = np.random.default_rng(1)
    tol = 1e-5 if dtype == "f32" else 1e-2
    for g in rng.choice(G, 24, replace=False):
        M, N, K = (int(x) for x in dims[g])
        a = Ah[offA[g]:offA[g + 1]].view(M, int(lda[g]))[:, :K].contiguous()
        b = Bh[offB[g]:offB[g + 1]].view(K, int(ldb[g]))[:, :N].contiguous()
        assert rel_fro(Cs[g].cpu().numpy(), om.matmul(a, b, dtype)) <= tol, g


MIXED = [(64, 64), (128, 64), (64, 128), (128, 128)]
MIXED_BK = {"f32": 32, "bf16": 64}


def mixed_params(dtype, G, stage, programs=MIXED):
    return [pk.params(family=pk.PK_FAMILY_MFMA, bm=programs[g % len(programs)][0], bn=programs[g % len(programs)][1],
                      bk=MIXED_BK[dtype], wm=2, wn=2, variant=stage) for g in range(G)]


@pytest.mark.parametrize("dtype,stage", [("f32", 0), ("f32", pk.PK_MFMA_SINGLE), ("bf16", pk.PK_MFMA_SINGLE)])
def test_mixed_tiles_one_launch_bit_identical(table, dtype, stage):
    # every product its own tile program, all four of the mixed kernel's
    # programs in one plan: one launch, each product equal bit for bit to the
    # single-product launch of its program, and to the oracle
    dims, host, dev = make_groups(48, seed=17, dtype=dtype, aligned_every=2, hi=300)
    As, Bs, Cs = zip(*dev)
    ps = mixed_params(dtype, len(As), stage)
    plan = pk.pk_grouped_plan_create(table, dtype, As, Bs, Cs, params=ps)
    n_launch, tiles, chosen = plan.info()
    kernels = plan.kernels()
    say("%s stage %d mixed plan: %s, %d tiles" % (dtype, stage, kernels, tiles))
    # one launch per row form (aligned rows, element loads), each the mixed kernel
    assert n_launch == len(row_forms(dtype, dev)) == 2, kernels
    assert all(k.startswith("pk_grouped_mixed_%s" % dtype) for k in kernels), kernels
    assert sorted(k.endswith("_el") for k in kernels) == [False, True], kernels
    assert len({(c.bm, c.bn) for c in chosen}) == 4
    plan.run()
    torch.cuda.synchronize()
    tol = 1e-5 if dtype == "f32" else 1e-2
    for g, ((a, b), (ad, bd, cd)) in enumerate(zip(host, dev)):
        got = cd.cpu()
        assert not torch.isnan(got).any(), g
        assert rel_fro(got.numpy(), om.matmul(a, b, dtype)) <= tol, (g, dims[g])
        C1 = torch.empty_like(cd)
        pk.pk_matmul(table, chosen[g], dtype, ad, bd, C1)
        torch.cuda.synchronize()
        assert torch.equal(C1.cpu(), got), (g, dims[g], chosen[g])


def test_mixed_tiles_accumulate_visits_each_tile_once(table):
    dims, host, dev = make_groups(40, seed=19, dtype="f32", aligned_every=3, hi=280)
    As, Bs, Cs = zip(*dev)
    ps = mixed_params("f32", len(As), 0)
    pk.pk_matmul_batched(table, "f32", As, Bs, Cs, params=ps)
    torch.cuda.synchronize()
    first = [c.cpu().clone() for c in Cs]
    for c in Cs:
        c.zero_()
    plan = pk.pk_grouped_plan_create(table, "f32", As, Bs, Cs, params=ps, accumulate=True)
    assert plan.info()[0] == len(row_forms("f32", dev))
    plan.run()
    plan.run()
    torch.cuda.synchronize()
    for g, c in enumerate(Cs):
        assert not torch.isnan(first[g]).any()
        assert torch.allclose(c.cpu(), 2 * first[g], rtol=1e-6, atol=1e-6), g


def test_two_stage_counts_get_launches_of_their_own(table):
    # one mixed kernel runs one stage count: products given two programs of
    # different stage counts run as one launch per grouped instance
    dims, host, dev = make_groups(24, seed=23, dtype="f32", aligned_every=1, hi=300)
    As, Bs, Cs = zip(*dev)
    ps = mixed_params("f32", len(As), 0, programs=[(64, 64)])
    for g in range(0, len(ps), 3):
        ps[g] = pk.params(family=pk.PK_FAMILY_MFMA, bm=128, bn=128, bk=32, wm=2, wn=2, variant=pk.PK_MFMA_SINGLE)
    plan = pk.pk_grouped_plan_create(table, "f32", As, Bs, Cs, params=ps)
    kernels = plan.kernels()
    say("launches: %s" % kernels)
    assert sorted(kernels) == ["pk_grouped_f32_128x128x32_w2x2_st1", "pk_grouped_f32_64x64x32_w2x2_st2"]
    plan.run()
    torch.cuda.synchronize()
    for (a, b), (ad, bd, cd) in zip(host, dev):
        assert rel_fro(cd.cpu().numpy(), om.matmul(a, b, "f32")) <= 1e-5


def test_case_plan_is_one_launch_and_learned_is_refused(table):
    # aligned rows: one launch of the wide kernel; with some rows unaligned, a
    # second launch of its element-load twin runs those products
    dims, host, dev = make_groups(64, seed=29, dtype="f32", aligned_every=1, lo=16, hi=512)
    As, Bs, Cs = zip(*dev)
    plan = pk.pk_grouped_plan_create(table, "f32", As, Bs, Cs)
    assert plan.info()[0] == 1 and not plan.kernels()[0].endswith("_el"), plan.kernels()
    dims, host, dev = make_groups(64, seed=29, dtype="f32", aligned_every=2, lo=16, hi=512)
    As, Bs, Cs = zip(*dev)
    plan = pk.pk_grouped_plan_create(table, "f32", As, Bs, Cs)
    assert len(row_forms("f32", dev)) == 2
    assert plan.info()[0] == 2 and sorted(k.endswith("_el") for k in plan.kernels()) == [False, True], plan.kernels()
    plan.run()
    torch.cuda.synchronize()
    for (a, b), (ad, bd, cd) in zip(host, dev):
        assert rel_fro(cd.cpu().numpy(), om.matmul(a, b, "f32")) <= 1e-5
    with pytest.raises(pk.PkError) as e:
        pk.pk_grouped_plan_create(table, "f32", As, Bs, Cs, policy=pk.PK_POLICY_LEARNED)
    assert e.value.code == pk.PK_ERR_INVALID_ARG


def test_empty_and_k0_products_in_a_mixed_plan(table):
    shapes = [(0, 5, 7), (6, 0, 3), (40, 70, 0), (33, 65, 17), (1, 1, 1), (129, 130, 131)]
    As, Bs, Cs, refs = [], [], [], []
    for i, (M, N, K) in enumerate(shapes):
        a = inputs.uniform_f32((M, K), seed=300 + 2 * i)
        b = inputs.uniform_f32((K, N), seed=301 + 2 * i)
        As.append(a.cuda())
        Bs.append(b.cuda())
        Cs.append(torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda"))
        refs.append(om.matmul(a, b, "f32") if M * N > 0 else None)
    ps = mixed_params("f32", len(shapes), 0)
    pk.pk_matmul_batched(table, "f32", As, Bs, Cs, params=ps)
    torch.cuda.synchronize()
    for i, (M, N, K) in enumerate(shapes):
        if M * N == 0:
            continue
        got = Cs[i].cpu().numpy()
        if K == 0:
            assert np.all(got == 0.0)
        else:
            assert rel_fro(got, refs[i]) <= 1e-5, shapes[i]
