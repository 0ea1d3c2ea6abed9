"""Selection paths through the C ABI on the device, each pick run against the
oracle: pk_measure (the auto-tuning measurement), the EXHAUSTIVE policy, the
LEARNED policy with its measurement fallback forced and switched off, the
LEARNED picks at the sweep's largest and most lopsided shapes checked on
whole rows and columns, and the cost model's inference against the float64
network of the oracle.

Bars: int32 bit-exact; float32 relative Frobenius error <= 1e-5 against the
float64 oracle; bfloat16 inputs (float32 accumulate) <= 1e-2.
"""
import math
import sys

import numpy as np
import pytest
import torch

import oracle.matmul as om
import oracle.mlp as mlp
from paper_1801_04348_amd import pk
from tests import inputs

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 1e-2}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_fro(c, ref):
    c = np.asarray(c, dtype=np.float64)
    num = np.linalg.norm(c - ref)
    den = np.linalg.norm(ref)
    return 0.0 if num == 0 else (num / den if den > 0 else np.inf)


@pytest.fixture(scope="module")
def table():
    return pk.pk_case_table_build(0)


@pytest.fixture(scope="module")
def learned_table():
    t = pk.pk_case_table_build(0)
    assert set(pk.load_shipped_models(t)) == {"f32", "i32", "bf16"}
    return t


def operands(dtype, M, N, K, seed):
    if dtype == "i32":
        return inputs.small_int_i32((M, K), seed=seed), inputs.small_int_i32((K, N), seed=seed + 1)
    A = inputs.uniform_f32((M, K), seed=seed)
    B = inputs.uniform_f32((K, N), seed=seed + 1)
    if dtype == "bf16":
        A, B = inputs.bf16_bits(A), inputs.bf16_bits(B)
    return A, B


def out_tensor(dtype, M, N):
    if dtype == "i32":
        return torch.full((M, N), -123456789, dtype=torch.int32, device="cuda")
    return torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")


def check(table, p, dtype, A, B, ref, Ad=None, Bd=None):
    M, K = A.shape
    N = B.shape[1]
    C = out_tensor(dtype, M, N)
    pk.pk_matmul(table, p, dtype, A.cuda() if Ad is None else Ad, B.cuda() if Bd is None else Bd, C)
    torch.cuda.synchronize()
    got = C.cpu().numpy()
    name = pk.pk_kernel_name(table, p, dtype)
    if dtype == "i32":
        assert np.array_equal(got, ref), name
    else:
        err = rel_fro(got, ref)
        assert err <= TOL[dtype], (name, err)


def feasible_count(table, dtype, wide=True):
    """Points of the product families whose case-table lookup gives a leaf;
    on rows not aligned for 16-byte loads (wide False) without the MFMA
    programs that have no element-load form."""
    d = pk.pk_case_table_describe(table)
    names = {e["name"] for e in d["instances"]}
    n = 0
    for part in d["parts"]:
        if part["family"] in (pk.PK_FAMILY_VALU, pk.PK_FAMILY_VALU2, pk.PK_FAMILY_MFMA) and \
                part["dtype"] == pk.DTYPES[dtype]:
            for pt, leaf in zip(part["points"], part["first_leaf"]):
                if leaf < 0:
                    continue
                if part["family"] == pk.PK_FAMILY_MFMA and not wide:
                    st = 1 if part["solution"]["leaves"][leaf]["variant"] & pk.PK_MFMA_SINGLE else 2
                    name = "pk_mfma_%s_%dx%dx%d_w%dx%d_st%d" % ((dtype,) + tuple(pt) + (st,))
                    if name + "_el" not in names:
                        continue
                n += 1
    return n


SEL_SHAPES = [(300, 260, 200), (1000, 3000, 512)]


@pytest.mark.parametrize("dtype", ["f32", "i32", "bf16"])
@pytest.mark.parametrize("shape", SEL_SHAPES)
def test_measure_and_exhaustive_pick(table, dtype, shape):
    M, N, K = shape
    A, B = operands(dtype, M, N, K, seed=101)
    ref = om.matmul(A, B, dtype)
    Ad, Bd = A.cuda(), B.cuda()
    C = out_tensor(dtype, M, N)
    say("pk_measure %s %s" % (dtype, shape))
    res = pk.pk_measure(table, dtype, M, N, K, Ad, Bd, C)
    # every feasible (leaf, E) is timed: every point with a leaf is a
    # candidate (on unaligned rows, those MFMA programs that have an
    # element-load form), run whole and (MFMA programs, few tiles) split
    # along K
    whole = [p for p, _ in res if p.ks <= 1]
    wide = pk.packed_rows_wide(dtype, N, K)
    assert len(whole) == feasible_count(table, dtype, wide), (len(whole), feasible_count(table, dtype, wide))
    assert all(p.family == pk.PK_FAMILY_MFMA for p, _ in res if p.ks > 1)
    secs = np.array([s for _, s in res])
    assert np.all(np.isfinite(secs)) and np.all(secs > 0), secs
    # distinct (leaf, E) pairs; two of them may run one compiled program (a
    # point whose leaf reduces the granularity runs the s = 1 instance)
    keys = [tuple(sorted(p.as_dict().items())) for p, _ in res]
    assert len(set(keys)) == len(keys)
    names = [pk.pk_kernel_name(table, p, dtype) for p, _ in res]
    # the fastest measured candidate and the EXHAUSTIVE pick both compute the product
    fastest = res[int(np.argmin(secs))][0]
    check(table, fastest, dtype, A, B, ref, Ad, Bd)
    p = pk.pk_select(table, dtype, M, N, K, pk.PK_POLICY_EXHAUSTIVE)
    name = pk.pk_kernel_name(table, p, dtype)
    say("exhaustive pick %s (fastest measured %s)" % (name, pk.pk_kernel_name(table, fastest, dtype)))
    assert name in names
    check(table, p, dtype, A, B, ref, Ad, Bd)
    # the pick is cached for the table's lifetime: asking again returns it
    assert pk.pk_kernel_name(table, pk.pk_select(table, dtype, M, N, K, pk.PK_POLICY_EXHAUSTIVE), dtype) == name


LEARNED_SHAPES = {"f32": (1000, 3000, 512), "i32": (300, 260, 200), "bf16": (512, 384, 264)}


@pytest.mark.parametrize("dtype", ["f32", "i32", "bf16"])
def test_learned_fallback_forced_and_off(learned_table, dtype):
    t = learned_table
    M, N, K = LEARNED_SHAPES[dtype]
    A, B = operands(dtype, M, N, K, seed=111)
    ref = om.matmul(A, B, dtype)
    try:
        # margin 1: every candidate predicted within 2x of the best is timed
        pk.pk_case_table_set_learned_margin(t, 1.0)
        sel0, fb0 = pk.pk_case_table_learned_stats(t)
        meas0 = pk.pk_case_table_learned_measured(t)
        p = pk.pk_select(t, dtype, M, N, K, pk.PK_POLICY_LEARNED)
        sel1, fb1 = pk.pk_case_table_learned_stats(t)
        meas1 = pk.pk_case_table_learned_measured(t)
        say("%s forced fallback: pick %s, %d candidates timed" % (dtype, pk.pk_kernel_name(t, p, dtype),
                                                                  meas1 - meas0))
        assert (sel1, fb1) == (sel0 + 1, fb0 + 1)
        assert meas1 - meas0 >= 2
        check(t, p, dtype, A, B, ref)
        # margin 0: the model's own pick, no timing
        pk.pk_case_table_set_learned_margin(t, 0.0)
        q = pk.pk_select(t, dtype, M, N, K, pk.PK_POLICY_LEARNED)
        sel2, fb2 = pk.pk_case_table_learned_stats(t)
        assert (sel2, fb2) == (sel1 + 1, fb1)
        assert pk.pk_case_table_learned_measured(t) == meas1
        check(t, q, dtype, A, B, ref)
    finally:
        pk.pk_case_table_set_learned_margin(t, 0.05)


def _slices_check(A, B, C, rows, cols):
    """Whole rows and columns of C against the oracle: relative Frobenius
    error of each slice and the standard per-element bound
    |c - ref| <= K u / (1 - K u) sum_k |a_ik b_kj|."""
    K = A.shape[1]
    ku = K * 2.0 ** -24
    Aa, Ba = A.abs(), B.abs()
    for i in rows:
        ref = om.matmul(A[i:i + 1], B, "f32")[0]
        bound = ku / (1 - ku) * om.matmul(Aa[i:i + 1], Ba, "f32")[0]
        got = C[i].double().numpy()
        assert rel_fro(got, ref) <= TOL["f32"], ("row", i)
        assert np.all(np.abs(got - ref) <= bound), ("row", i)
    for j in cols:
        ref = om.matmul(A, B[:, j:j + 1].contiguous(), "f32")[:, 0]
        bound = ku / (1 - ku) * om.matmul(Aa, Ba[:, j:j + 1].contiguous(), "f32")[:, 0]
        got = C[:, j].double().numpy()
        assert rel_fro(got, ref) <= TOL["f32"], ("column", j)
        assert np.all(np.abs(got - ref) <= bound), ("column", j)


@pytest.mark.parametrize("shape", [(8192, 8192, 8192), (512, 512, 8192), (8192, 3000, 4096), (3000, 8192, 1000)])
def test_full_size_learned_pick_rows_and_columns(learned_table, shape):
    t = learned_table
    M, N, K = shape
    A = inputs.uniform_f32((M, K), seed=121)
    B = inputs.uniform_f32((K, N), seed=122)
    p = pk.pk_select(t, "f32", M, N, K, pk.PK_POLICY_LEARNED)
    say("full size %s LEARNED pick %s" % (shape, pk.pk_kernel_name(t, p, "f32")))
    C = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    pk.pk_matmul(t, p, "f32", A.cuda(), B.cuda(), C)
    torch.cuda.synchronize()
    Ch = C.cpu()
    assert not torch.isnan(Ch).any()
    # first and last rows and columns (edge tiles) and one in the middle
    _slices_check(A, B, Ch, rows=[0, M // 2 + 1, M - 1], cols=[0, N // 2 + 3, N - 1])


def _read_model(path):
    """Parameters and standardisation of a model file (text: keyword lines,
    then every parameter value after the "params <count>" line)."""
    lines = open(path).read().splitlines()
    at = next(i for i, ln in enumerate(lines) if ln.startswith("params"))
    vals = {ln.split()[0]: ln.split()[1:] for ln in lines[:at + 1] if ln.strip()}
    params = np.array([float(v) for ln in lines[at + 1:] for v in ln.split()], dtype=np.float64)
    assert params.size == int(vals["params"][0]) == mlp.NPARAM
    xmean = np.array([float(v) for v in vals["xmean"]])
    xstd = np.array([float(v) for v in vals["xstd"]])
    ymean, ystd = (float(v) for v in vals["y"])
    return params, xmean, xstd, ymean, ystd


def _has_split_form(table, p, dtype):
    # the single-stage float32 programs of 512 work-items have none
    try:
        pk.pk_kernel_name(table, p, dtype)
    except pk.PkError:
        return False
    return True


@pytest.mark.parametrize("dtype", ["f32", "i32", "bf16"])
def test_costmodel_inference_matches_oracle_network(learned_table, dtype):
    import os
    path = os.path.join(os.path.dirname(pk.__file__), "data", "costmodel_%s_gfx950.txt" % dtype)
    cm = pk.pk_costmodel_load(path)
    params, xmean, xstd, ymean, ystd = _read_model(path)
    assert np.array_equal(params.astype(np.float32), cm.params())
    # feature rows of real candidates (every point of the dtype's product
    # families at 40 random shapes), then random rows around them
    rng = np.random.default_rng(3)
    d = pk.pk_case_table_describe(learned_table)
    rows = []
    for (M, N, K) in inputs.log_uniform_shapes(40, seed=7):
        for part in d["parts"]:
            fam = part["family"]
            if fam not in (pk.PK_FAMILY_VALU, pk.PK_FAMILY_VALU2, pk.PK_FAMILY_MFMA) or \
                    part["dtype"] != pk.DTYPES[dtype]:
                continue
            for pt, leaf in zip(part["points"], part["first_leaf"]):
                if leaf < 0:
                    continue
                if fam == pk.PK_FAMILY_VALU:
                    p = pk.params(bx=pt[0], by=pt[1], s=pt[2])
                elif fam == pk.PK_FAMILY_VALU2:
                    p = pk.params(family=fam, bx=pt[0], by=pt[1], s=pt[2], sy=pt[3], bk=pt[4])
                else:   # split along K in some rows (where the program has a split form)
                    ks = int(rng.choice([0, 2, 4])) if 64 * pt[3] * pt[4] <= 512 else 0
                    p = pk.params(family=fam, bm=pt[0], bn=pt[1], bk=pt[2], wm=pt[3], wn=pt[4], ks=ks)
                    if ks and not _has_split_form(learned_table, p, dtype):
                        p.ks = 0
                rows.append(pk.pk_features(learned_table, p, dtype, int(M), int(N), int(K),
                                           wide=bool(rng.integers(0, 2))))
    X = np.array(rows, dtype=np.float32)
    X = np.concatenate([X, (X[rng.integers(0, len(X), 200)] + rng.normal(scale=0.3, size=(200, mlp.IN)))
                        .astype(np.float32)])
    say("%s: %d feature rows" % (dtype, len(X)))
    got = cm.predict(X)
    # the oracle: standardise in float64, the network's forward, undo the
    # target standardisation
    Xs = (X.astype(np.float64) - xmean.astype(np.float32)) / xstd.astype(np.float32)
    y, _ = mlp.forward(mlp.unflatten(params.astype(np.float32).astype(np.float64)), Xs)
    ref = y * np.float32(ystd) + np.float32(ymean)
    # float32 inference: a few roundings of the magnitudes that enter
    # (ln seconds of order 10): 1e-4 absolute is 0.01 % of a predicted time
    err = np.abs(got.astype(np.float64) - ref)
    assert np.max(err) <= 1e-4, (np.max(err), int(np.argmax(err)))


def test_twinless_program_on_unaligned_rows_runs_the_case_choice():
    # on a machine whose block register budget admits the 1024-work-item
    # bfloat16 256 x 256 x 64 tile, pk_select picks it for a large product;
    # that program has no element-load form, so given unaligned rows
    # pk_matmul runs the CASE choice for those operands instead
    m = pk.pk_machine_query(0)
    m.regs_block = max(m.regs_block, 131072)
    t = pk.pk_case_table_build(0, m)
    p = pk.params(family=pk.PK_FAMILY_MFMA, bm=256, bn=256, bk=64, wm=4, wn=4)
    assert pk.pk_kernel_name(t, p, "bf16").startswith("pk_mfma_bf16_256x256x64")
    M, N, K = 37, 19, 45                     # packed: lda = 45, ldb = 19, unaligned rows
    A, B = operands("bf16", M, N, K, seed=131)
    ref = om.matmul(A, B, "bf16")
    check(t, p, "bf16", A, B, ref)
