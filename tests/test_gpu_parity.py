"""Parity of every HIP leaf with the CPU oracle, through the C ABI.

Bars: int32 bit-exact; float32 relative Frobenius error <= 1e-5 against the
float64 oracle; bfloat16 inputs (float32 accumulate) <= 1e-2.  Float inputs
that are small integers must come out bit-exact in every leaf, as every
partial sum is then an exact integer below 2^24.
"""
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
BF16_TOL = 1e-2
VALU_VARIANTS = (0, pk.PK_VALU_GRAN, pk.PK_VALU_GRAN | pk.PK_VALU_NOLDS, pk.PK_VALU_NOLDS)
MFMA_VARIANTS = (0, pk.PK_MFMA_SINGLE)


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
def desc(table):
    return pk.pk_case_table_describe(table)


def dev(t):
    return t.to("cuda")


@pytest.fixture(scope="module")
def fit(desc):
    """fit(family, dtype, variant, point): does the program fit this device,
    by the oracle's own resource derivation?"""
    inst = en.InstanceData(desc["instances"])
    m = desc["machine"]

    def f(family, dtype, variant, point):
        return en.fits(inst, family, pk.DTYPES[dtype], variant, tuple(point), m["lds_block"], m["regs_block"],
                       m["max_threads_block"])
    return f


def forced(table, fit, family, dtype, variant, point, p, A, B, M, N, **kw):
    """Runs a forced variant where it fits; elsewhere checks it is refused."""
    if fit(family, dtype, variant, point):
        return run(table, p, dtype, A, B, M, N, **kw)
    with pytest.raises(pk.PkError) as e:
        run(table, p, dtype, A, B, M, N, **kw)
    assert e.value.code == pk.PK_ERR_NO_FEASIBLE_BRANCH
    return None


def run(table, p, dtype, A, B, M, N, accumulate=False, C0=None, out_dtype=torch.float32):
    if C0 is not None:
        C = C0.clone()
    elif out_dtype == torch.int32:
        C = torch.full((M, N), -123456789, dtype=torch.int32, device="cuda")
    else:
        C = torch.full((M, N), float("nan"), dtype=out_dtype, device="cuda")
    pk.pk_matmul(table, p, dtype, A, B, C, accumulate=accumulate)
    torch.cuda.synchronize()
    return C.cpu()


def test_machine_query_matches_runtime_props():
    # the library reads hipDeviceProp_t through the HIP runtime loaded in this
    # process; torch reads the same structure independently
    m = pk.pk_machine_query(0)
    tp = torch.cuda.get_device_properties(0)
    say("machine:", m.as_dict())
    assert m.wave == 64 == getattr(tp, "warp_size", 64)
    assert m.cu_count == tp.multi_processor_count
    if hasattr(tp, "shared_memory_per_block"):
        assert m.lds_block == tp.shared_memory_per_block
    if hasattr(tp, "regs_per_multiprocessor"):
        assert m.regs_cu == tp.regs_per_multiprocessor
    if hasattr(tp, "max_threads_per_multi_processor"):
        assert m.max_threads_cu == tp.max_threads_per_multi_processor
    assert m.max_threads_block == 1024
    assert m.arch.decode().startswith("gfx950")


# ---------------------------------------------------------------- f32 256^3
F32_256_E = [(bx, by, s) for bx in (8, 16, 32) for by in (8, 16, 32) for s in (1, 2, 4)]


@pytest.fixture(scope="module")
def f32_256():
    A = inputs.uniform_f32((256, 256), seed=0)
    B = inputs.uniform_f32((256, 256), seed=1)
    return dev(A), dev(B), om.matmul(A, B, "f32")


@pytest.mark.parametrize("E", F32_256_E)
def test_f32_256_every_leaf_and_variant(table, fit, f32_256, E):
    A, B, ref = f32_256
    bx, by, s = E
    leaf, var = pk.pk_case_table_lookup(table, "f32", pk.params(bx=bx, by=by, s=s))
    say("f32 256^3 E=%s leaf=%d variant=%d" % (E, leaf, var))
    C = run(table, pk.params(leaf=leaf, bx=bx, by=by, s=s), "f32", A, B, 256, 256)
    assert rel_fro(C.numpy(), ref) <= F32_TOL
    for v in VALU_VARIANTS:  # forced: every program where it fits
        C = forced(table, fit, 0, "f32", v, E, pk.params(variant=v, bx=bx, by=by, s=s), A, B, 256, 256)
        assert C is None or rel_fro(C.numpy(), ref) <= F32_TOL, (E, v)


# ---------------------------------------------------------------- i32 1024^3
I32_1024_B = (4, 8, 16, 32)


@pytest.fixture(scope="module")
def i32_1024():
    A = inputs.small_int_i32((1024, 1024), seed=0)
    B = inputs.small_int_i32((1024, 1024), seed=1)
    return dev(A), dev(B), om.matmul(A, B, "i32")


@pytest.mark.parametrize("bx", I32_1024_B)
@pytest.mark.parametrize("by", I32_1024_B)
def test_i32_1024_every_leaf_and_variant_bit_exact(table, fit, i32_1024, bx, by):
    A, B, ref = i32_1024
    for s in (1, 2, 4, 8):
        leaf, var = pk.pk_case_table_lookup(table, "i32", pk.params(bx=bx, by=by, s=s))
        say("i32 1024^3 E=(%d,%d,%d) leaf=%d variant=%d" % (bx, by, s, leaf, var))
        C = run(table, pk.params(leaf=leaf, bx=bx, by=by, s=s), "i32", A, B, 1024, 1024, out_dtype=torch.int32)
        assert np.array_equal(C.numpy(), ref)
        for v in VALU_VARIANTS:
            C = forced(table, fit, 0, "i32", v, (bx, by, s), pk.params(variant=v, bx=bx, by=by, s=s), A, B,
                       1024, 1024, out_dtype=torch.int32)
            assert C is None or np.array_equal(C.numpy(), ref), (bx, by, s, v)


def test_i32_full_range_wraps(table, fit):
    A = inputs.full_range_i32((77, 130), seed=5)
    B = inputs.full_range_i32((130, 91), seed=6)
    ref = om.matmul(A, B, "i32")
    for E in [(4, 4, 1), (16, 8, 4), (32, 32, 8), (8, 32, 2)]:
        for v in VALU_VARIANTS:
            C = forced(table, fit, 0, "i32", v, E, pk.params(variant=v, bx=E[0], by=E[1], s=E[2]), dev(A), dev(B), 77, 91,
                    out_dtype=torch.int32)
            assert C is None or np.array_equal(C.numpy(), ref), (E, v)


# ---------------------------------------------------------------- MFMA leaves
def twinless(desc, dtype, pt, v):
    """The MFMA program has no element-load twin among the compiled instances."""
    name = "pk_mfma_%s_%dx%dx%d_w%dx%d_st%d" % ((dtype,) + tuple(pt) + (1 if v & pk.PK_MFMA_SINGLE else 2,))
    names = {e["name"] for e in desc["instances"]}
    assert name in names, name
    return name + "_el" not in names


def mfma_points(desc, dtype):
    pts = []
    for part in desc["parts"]:
        if part["family"] == pk.PK_FAMILY_MFMA and part["dtype"] == pk.DTYPES[dtype]:
            pts = [tuple(p) for p in part["points"]]
    return pts


def mfma_params(pt, variant):
    bm, bn, bk, wm, wn = pt
    return pk.params(family=pk.PK_FAMILY_MFMA, variant=variant, bm=bm, bn=bn, bk=bk, wm=wm, wn=wn)


@pytest.mark.parametrize("shape", [(300, 260, 200), (512, 512, 512), (129, 65, 33), (1, 1, 1)])
def test_mfma_f32_every_instance(table, fit, desc, shape):
    M, N, K = shape
    A = inputs.uniform_f32((M, K), seed=11)
    B = inputs.uniform_f32((K, N), seed=12)
    ref = om.matmul(A, B, "f32")
    Ad, Bd = dev(A), dev(B)
    # K = 1 or 33 leaves rows unaligned for 16-byte loads: pad lda
    if K % 4:
        Kp = (K + 3) // 4 * 4
        Ap = torch.zeros((M, Kp), dtype=torch.float32)
        Ap[:, :K] = A
        Ad = dev(Ap)[:, :K]
    if N % 4:
        Np = (N + 3) // 4 * 4
        Bp = torch.zeros((K, Np), dtype=torch.float32)
        Bp[:, :N] = B
        Bd = dev(Bp)[:, :N]
    for pt in mfma_points(desc, "f32"):
        for v in MFMA_VARIANTS:
            say("mfma f32 %s %s variant %d" % (shape, pt, v))
            C = forced(table, fit, 1, "f32", v, pt, mfma_params(pt, v), Ad, Bd, M, N)
            assert C is None or rel_fro(C.numpy(), ref) <= F32_TOL, (pt, v)


@pytest.mark.parametrize("shape", [(300, 260, 200), (512, 512, 512), (129, 66, 40)])
def test_mfma_bf16_every_instance(table, fit, desc, shape):
    M, N, K = shape
    A = inputs.bf16_bits(inputs.uniform_f32((M, K), seed=21))
    B = inputs.bf16_bits(inputs.uniform_f32((K, N), seed=22))
    ref = om.matmul(A, B, "bf16")
    for pt in mfma_points(desc, "bf16"):
        for v in MFMA_VARIANTS:
            say("mfma bf16 %s %s variant %d" % (shape, pt, v))
            C = forced(table, fit, 1, "bf16", v, pt, mfma_params(pt, v), dev(A), dev(B), M, N)
            if C is None:
                continue
            err = rel_fro(C.numpy(), ref)
            assert err <= BF16_TOL, (pt, v, err)
            assert err <= 1e-5, (pt, v, err)  # float32 accumulation of exact products


def test_small_integers_bit_exact_all_families(table, fit, desc):
    M, N, K = 200, 136, 1000
    A = inputs.small_int_f32((M, K), seed=31)
    B = inputs.small_int_f32((K, N), seed=32)
    ref = om.matmul(A, B, "f32")
    for E in [(4, 4, 1), (16, 8, 4), (32, 32, 8), (8, 16, 2)]:
        for v in VALU_VARIANTS:
            C = forced(table, fit, 0, "f32", v, E, pk.params(variant=v, bx=E[0], by=E[1], s=E[2]), dev(A), dev(B), M, N)
            assert C is None or np.array_equal(C.numpy().astype(np.float64), ref), (E, v)
    for pt in mfma_points(desc, "f32"):
        for v in MFMA_VARIANTS:
            C = forced(table, fit, 1, "f32", v, pt, mfma_params(pt, v), dev(A), dev(B), M, N)
            assert C is None or np.array_equal(C.numpy().astype(np.float64), ref), (pt, v)
    Ab, Bb = inputs.bf16_bits(A), inputs.bf16_bits(B)
    for pt in mfma_points(desc, "bf16"):
        for v in MFMA_VARIANTS:
            C = forced(table, fit, 1, "bf16", v, pt, mfma_params(pt, v), dev(Ab), dev(Bb), M, N)
            assert C is None or np.array_equal(C.numpy().astype(np.float64), ref), (pt, v)


def test_identity_returns_b(table, fit, desc):
    n = 160
    B = inputs.uniform_f32((n, 96), seed=41)
    I = torch.eye(n, dtype=torch.float32)
    for E in [(8, 8, 1), (32, 16, 4)]:
        for v in VALU_VARIANTS:
            C = forced(table, fit, 0, "f32", v, E, pk.params(variant=v, bx=E[0], by=E[1], s=E[2]), dev(I), dev(B), n, 96)
            assert C is None or torch.equal(C, B)
    for pt in mfma_points(desc, "f32"):
        C = forced(table, fit, 1, "f32", 0, pt, mfma_params(pt, 0), dev(I), dev(B), n, 96)
        assert C is None or torch.equal(C, B), pt


def test_accumulate_mode(table, desc):
    M, N, K = 190, 200, 70
    A = inputs.uniform_f32((M, K), seed=51)
    B = inputs.uniform_f32((K, 200), seed=52)
    C0 = inputs.uniform_f32((M, N), seed=53)
    ref = om.matmul(A, B, "f32", Cin=C0.double().numpy())
    for p in [pk.params(variant=0, bx=16, by=8, s=4), pk.params(variant=pk.PK_VALU_NOLDS, bx=8, by=8, s=2)] + \
             [mfma_params(pt, 0) for pt in mfma_points(desc, "f32")[:3]]:
        Kp = (K + 3) // 4 * 4
        Ap = torch.zeros((M, Kp))
        Ap[:, :K] = A
        C = run(table, p, "f32", dev(Ap)[:, :K], dev(B), M, N, accumulate=True, C0=dev(C0))
        assert rel_fro(C.numpy(), ref) <= F32_TOL, p
    Ai = inputs.full_range_i32((M, K), seed=54)
    Bi = inputs.full_range_i32((K, N), seed=55)
    Ci = inputs.full_range_i32((M, N), seed=56)
    refi = om.matmul(Ai, Bi, "i32", Cin=Ci.numpy())
    C = run(table, pk.params(variant=0, bx=16, by=16, s=2), "i32", dev(Ai), dev(Bi), M, N, accumulate=True,
            C0=dev(Ci))
    assert np.array_equal(C.numpy(), refi)


def test_every_tile_visited_once(table, desc, fit):
    # NaN sentinels must all be overwritten; accumulating twice into zeros
    # must give exactly twice the product (a tile visited twice would not)
    M, N, K = 333, 268, 64
    A = dev(inputs.small_int_f32((M, K), seed=61))
    B = dev(inputs.small_int_f32((K, N), seed=62))
    ps = [pk.params(variant=v, bx=bx, by=by, s=s) for v in VALU_VARIANTS for (bx, by, s) in [(4, 8, 8), (32, 4, 2)]
          if fit(0, "f32", v, (bx, by, s))]
    ps += [mfma_params(pt, v) for pt in mfma_points(desc, "f32") for v in MFMA_VARIANTS if fit(1, "f32", v, pt)]
    for p in ps:
        C = run(table, p, "f32", A, B, M, N)
        assert not torch.isnan(C).any(), p
        Z = torch.zeros((M, N), device="cuda")
        pk.pk_matmul(table, p, "f32", A, B, Z, accumulate=True)
        pk.pk_matmul(table, p, "f32", A, B, Z, accumulate=True)
        torch.cuda.synchronize()
        assert torch.equal(Z.cpu(), 2 * C), p


@pytest.mark.parametrize("M,N,K", [(m, n, k) for m in (1, 2, 7) for n in (1, 3, 9) for k in (0, 1, 5, 9)])
def test_tiny_shapes(table, M, N, K):
    A = inputs.uniform_f32((M, K), seed=M + 10 * N + 100 * K)
    B = inputs.uniform_f32((K, N), seed=M + 10 * N + 100 * K + 1)
    ref = om.matmul(A, B, "f32")
    for p in [pk.params(variant=0, bx=4, by=4, s=2), pk.params(variant=3, bx=32, by=8, s=1), None]:
        C = run(table, p, "f32", dev(A), dev(B), M, N)
        assert rel_fro(C.numpy(), ref) <= F32_TOL, (p, M, N, K)
    # K == 0 with accumulate leaves C unchanged
    C0 = inputs.uniform_f32((M, N), seed=7)
    if K == 0:
        C = run(table, None, "f32", dev(A), dev(B), M, N, accumulate=True, C0=dev(C0))
        assert torch.equal(C, C0)


def test_empty_output_is_noop(table):
    A = torch.zeros((0, 5), device="cuda")
    B = torch.zeros((5, 4), device="cuda")
    C = torch.zeros((0, 4), device="cuda")
    pk.pk_matmul(table, None, "f32", A, B, C)
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_unaligned_rows_take_element_loads(table, fit, desc, dtype):
    # operands one element off 16-byte alignment with odd leading dimensions:
    # every MFMA program reads them element by element, with the same tile
    # arithmetic, so the result is bit-identical to the aligned run
    M, N, K = 131, 70, 45
    if dtype == "f32":
        A = inputs.uniform_f32((M, K), seed=71)
        B = inputs.uniform_f32((K, N), seed=72)
    else:
        A = inputs.bf16_bits(inputs.uniform_f32((M, K), seed=71))
        B = inputs.bf16_bits(inputs.uniform_f32((K, N), seed=72))
    ref = om.matmul(A, B, dtype)
    Au = dev(torch.cat([A.new_zeros((M, 1)), A, A.new_zeros((M, 2))], dim=1))[:, 1:K + 1]   # lda = K + 3
    Bu = dev(torch.cat([B.new_zeros((K, 1)), B, B.new_zeros((K, 2))], dim=1))[:, 1:N + 1]   # ldb = N + 3
    Kp, Np = (K + 7) // 8 * 8, (N + 7) // 8 * 8
    Aa = dev(torch.cat([A, A.new_zeros((M, Kp - K))], dim=1))[:, :K]
    Ba = dev(torch.cat([B, B.new_zeros((K, Np - N))], dim=1))[:, :N]
    tol = F32_TOL if dtype == "f32" else BF16_TOL
    for pt in mfma_points(desc, dtype):
        for v in MFMA_VARIANTS:
            say("mfma %s unaligned %s variant %d" % (dtype, pt, v))
            if twinless(desc, dtype, pt, v) and fit(1, dtype, v, pt):
                # no element-load form of this tile: the CASE choice for these operands runs
                C = run(table, mfma_params(pt, v), dtype, Au, Bu, M, N)
                assert rel_fro(C.numpy(), ref) <= tol, (pt, v)
                continue
            Cu = forced(table, fit, 1, dtype, v, pt, mfma_params(pt, v), Au, Bu, M, N)
            if Cu is None:
                continue
            Ca = forced(table, fit, 1, dtype, v, pt, mfma_params(pt, v), Aa, Ba, M, N)
            assert rel_fro(Cu.numpy(), ref) <= tol, (pt, v)
            assert np.array_equal(Cu.numpy(), Ca.numpy()), (pt, v)
    C = run(table, None, dtype, Au, Bu, M, N)            # the CASE pick on these operands
    assert rel_fro(C.numpy(), ref) <= tol


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (3, 9, 5), (7, 1, 33), (65, 3, 70)])
def test_tiny_unaligned_shapes_every_twin(table, fit, desc, dtype, M, N, K):
    # packed operands of these shapes have unaligned rows, so every MFMA
    # program runs as its element-load twin: every step is an edge step
    # (rows and columns clamped, k beyond K read from the zero block); a plain
    # and an accumulating run against the oracle
    A = inputs.uniform_f32((M, K), seed=91 + M)
    B = inputs.uniform_f32((K, N), seed=92 + N)
    if dtype == "bf16":
        A, B = inputs.bf16_bits(A), inputs.bf16_bits(B)
    C0 = inputs.uniform_f32((M, N), seed=93)
    ref = om.matmul(A, B, dtype)
    ref_acc = om.matmul(A, B, dtype, Cin=C0.double().numpy())
    tol = F32_TOL if dtype == "f32" else BF16_TOL
    for pt in mfma_points(desc, dtype):
        for v in MFMA_VARIANTS:
            if not fit(1, dtype, v, pt) or twinless(desc, dtype, pt, v):
                continue
            say("mfma %s twin %s variant %d on %dx%dx%d" % (dtype, pt, v, M, N, K))
            C = run(table, mfma_params(pt, v), dtype, dev(A), dev(B), M, N)
            assert rel_fro(C.numpy(), ref) <= tol, (pt, v)
            C = run(table, mfma_params(pt, v), dtype, dev(A), dev(B), M, N, accumulate=True, C0=dev(C0))
            assert rel_fro(C.numpy(), ref_acc) <= tol, (pt, v)


# ---------------------------------------------------------------- full sizes, CASE pick (as benchmarked)
def sampled_check(A, B, C, dtype, nsamp=48, seed=0):
    """Sampled elements against the oracle, one by one: the relative RMS error
    over the samples (an estimate of the relative Frobenius error) and the
    standard worst-case bound |c - ref| <= K u sum_k |a_ik b_kj| per element."""
    rng = np.random.default_rng(seed)
    M, K = A.shape
    N = B.shape[1]
    rows = rng.integers(0, M, nsamp)
    cols = rng.integers(0, N, nsamp)
    An = A.numpy()
    Bn = B.numpy()
    errs, refs = [], []
    for i, j in zip(rows, cols):
        ref = om.dot(An, Bn, int(i), int(j), dtype)
        c = float(C[i, j])
        if dtype == "bf16":
            a = inputs.bf16_bits_to_f32(A[i]).double().numpy()
            b = inputs.bf16_bits_to_f32(B[:, j].contiguous()).double().numpy()
        else:
            a = An[i].astype(np.float64)
            b = Bn[:, j].astype(np.float64)
        ku = K * 2.0 ** -24
        bound = ku / (1.0 - ku) * np.sum(np.abs(a * b))
        assert abs(c - ref) <= bound, (i, j, c, ref, bound)
        errs.append(c - ref)
        refs.append(ref)
    return float(np.sqrt(np.mean(np.square(errs))) / np.sqrt(np.mean(np.square(refs))))


@pytest.mark.parametrize("shape", [(8192, 8192, 8192), (1000, 3000, 8192), (3000, 512, 1000), (4096, 4096, 4096)])
def test_full_size_case_pick_sampled(table, shape):
    M, N, K = shape
    A = inputs.uniform_f32((M, K), seed=81)
    B = inputs.uniform_f32((K, N), seed=82)
    p = pk.pk_select(table, "f32", M, N, K)
    say("full size %s pick %s" % (shape, p))
    C = run(table, None, "f32", dev(A), dev(B), M, N)
    assert not torch.isnan(C).any()
    assert sampled_check(A, B, C, "f32") <= F32_TOL
