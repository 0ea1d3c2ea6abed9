"""The cost model's kernels against the float64 oracle (GPU), and its host
side: feature values and the model file (CPU)."""
import math
import os

import numpy as np
import pytest

import oracle.matmul as om
import oracle.mlp as mlp
from paper_1801_04348_amd import pk
from tests import inputs, machines


def _write_model(path, params, xmean, xstd, ymean, ystd, machine="m"):
    with open(path, "w") as f:
        f.write("pk-costmodel 1\nfeatures %d\nmachine %s\nepochs 0\nloss 0\n" % (mlp.IN, machine))
        f.write("xmean " + " ".join("%.9g" % v for v in xmean) + "\n")
        f.write("xstd " + " ".join("%.9g" % v for v in xstd) + "\n")
        f.write("y %.9g %.9g\nparams %d\n" % (ymean, ystd, len(params)))
        f.write(" ".join("%.9g" % v for v in params) + "\n")


def test_model_file_roundtrip(tmp_path):
    p = mlp.init_params(3).astype(np.float32)
    path = str(tmp_path / "m.txt")
    _write_model(path, p, np.zeros(mlp.IN), np.ones(mlp.IN), 0.5, 2.0)
    cm = pk.pk_costmodel_load(path)
    assert np.array_equal(cm.params(), p)
    assert cm.machine() == "m"
    path2 = str(tmp_path / "m2.txt")
    cm.save(path2)
    assert np.array_equal(pk.pk_costmodel_load(path2).params(), p)


def test_model_dtype_roundtrip_and_per_type_selection(tmp_path):
    # a file without a dtype line is float32; set_dtype survives save/load
    path = str(tmp_path / "m.txt")
    m = machines.gfx950()
    t = pk.pk_case_table_build(0, m)
    desc_machine = pk.pk_case_table_describe(t)["machine"]
    finger = "%s/cu%d/lds%d/regs%d/thr%d/clk%d" % (desc_machine["arch"], desc_machine["cu_count"],
                                                  desc_machine["lds_block"], desc_machine["regs_block"],
                                                  desc_machine["max_threads_block"], desc_machine["clock_khz"])
    _write_model(path, mlp.init_params(3).astype(np.float32), np.zeros(mlp.IN), np.ones(mlp.IN), 0.0, 1.0,
                 machine=finger)
    cm = pk.pk_costmodel_load(path)
    assert cm.dtype() == "f32"
    cm.set_dtype("i32")
    path2 = str(tmp_path / "m2.txt")
    cm.save(path2)
    assert "dtype i32" in open(path2).read()
    cm2 = pk.pk_costmodel_load(path2)
    assert cm2.dtype() == "i32"
    # the table holds a model per element type: with only an int32 model, a
    # float32 LEARNED selection is the CASE pick with PK_ERR_COST_MODEL
    pk.pk_case_table_set_costmodel(t, cm2)
    with pytest.raises(pk.PkError) as e:
        pk.pk_select(t, "f32", 1000, 1000, 1000, pk.PK_POLICY_LEARNED)
    assert e.value.code == pk.PK_ERR_COST_MODEL
    p = pk.pk_select(t, "f32", 1000, 1000, 1000, pk.PK_POLICY_LEARNED, allow_fallback=True)
    assert pk.pk_kernel_name(t, p, "f32") == pk.pk_kernel_name(t, pk.pk_select(t, "f32", 1000, 1000, 1000), "f32")
    with open(path2.replace("m2", "bad"), "w") as f:
        f.write(open(path2).read().replace("dtype i32", "dtype f64"))
    with pytest.raises(pk.PkError) as e:
        pk.pk_costmodel_load(path2.replace("m2", "bad"))
    assert e.value.code == pk.PK_ERR_COST_MODEL


def test_model_file_rejects_wrong_sizes(tmp_path):
    path = str(tmp_path / "bad.txt")
    _write_model(path, np.zeros(10, np.float32), np.zeros(mlp.IN), np.ones(mlp.IN), 0, 1)
    with pytest.raises(pk.PkError) as e:
        pk.pk_costmodel_load(path)
    assert e.value.code == pk.PK_ERR_COST_MODEL


def test_model_for_other_machine_refused(tmp_path):
    path = str(tmp_path / "m.txt")
    _write_model(path, mlp.init_params(1).astype(np.float32), np.zeros(mlp.IN), np.ones(mlp.IN), 0, 1,
                 machine="someone-else")
    t = pk.pk_case_table_build(0, machines.gfx950())
    with pytest.raises(pk.PkError) as e:
        pk.pk_case_table_set_costmodel(t, pk.pk_costmodel_load(path))
    assert e.value.code == pk.PK_ERR_COST_MODEL


def test_features_by_hand():
    m = machines.gfx950()
    t = pk.pk_case_table_build(0, m)
    p = pk.params(family=pk.PK_FAMILY_MFMA, bm=128, bn=128, bk=32, wm=2, wn=2)
    M, N, K = 1000, 3000, 512
    f = pk.pk_features(t, p, "f32", M, N, K)
    d = pk.pk_case_table_describe(t)
    inst = [e for e in d["instances"] if e["name"] == pk.pk_kernel_name(t, p, "f32")][0]
    # occupancy by hand: LDS, threads, registers and the slot limit
    per_lane = -(-(-(-inst["vgpr"] // 4) * 4 + inst["agpr"]) // 8) * 8
    regs = per_lane * 64 * 4
    occ = min(m.max_blocks_cu, m.lds_cu // inst["lds_bytes"], m.max_threads_cu // 256, m.regs_cu // regs)
    tiles = math.ceil(M / 128) * math.ceil(N / 128)
    slots = m.cu_count * occ
    rounds = math.ceil(tiles / slots)
    want = [math.log(M), math.log(N), math.log(K), math.log(128), math.log(128), math.log(128 * 128 / 256),
            inst["lds_bytes"] / 65536, min(1.0, occ * 4 / (m.max_threads_cu / 64)),
            M * N / (math.ceil(M / 128) * 128 * math.ceil(N / 128) * 128), tiles / (rounds * slots), 1.0, 0.0,
            math.log(pk.pk_estimate(t, p, "f32", M, N, K))]
    assert np.allclose(f, want, rtol=1e-6, atol=1e-7), (f, want)
    f0 = pk.pk_features(t, p, "f32", M, N, K, wide=False)
    assert f0[10] == 0.0 and np.array_equal(f0[:10], f[:10])
    assert np.isclose(f0[12], math.log(pk.pk_estimate(t, p, "f32", M, N, K, wide=False)), rtol=1e-6)
    # split along K in 4: four workgroups per tile, ln 4 as feature 11
    p.ks = 4
    f4 = pk.pk_features(t, p, "f32", M, N, K)
    rounds4 = math.ceil(4 * tiles / slots)
    assert np.isclose(f4[9], 4 * tiles / (rounds4 * slots)) and np.isclose(f4[11], math.log(4))
    assert np.isclose(f4[12], math.log(pk.pk_estimate(t, p, "f32", M, N, K)), rtol=1e-6) and f4[12] != f[12]
    assert np.array_equal(np.delete(f4, [9, 11, 12]), np.delete(f, [9, 11, 12]))
    assert pk.packed_rows_wide("f32", 3000, 512) and not pk.packed_rows_wide("f32", 3000, 513)
    assert pk.packed_rows_wide("bf16", 3000, 512) and not pk.packed_rows_wide("bf16", 3001, 512)
    # bfloat16 rows of B need 16 bytes too: N a multiple of 8 elements
    assert not pk.packed_rows_wide("bf16", 3004, 512) and not pk.packed_rows_wide("bf16", 3000, 516)


@pytest.mark.gpu
def test_gradient_matches_float64_oracle():
    rng = np.random.default_rng(0)
    n = 1000  # 15 full workgroups of 64 rows and a ragged tail of 40
    X = rng.normal(size=(n, mlp.IN)).astype(np.float32)
    t = rng.normal(size=n).astype(np.float32)
    P = mlp.init_params(7).astype(np.float32)
    P[mlp.IN * 64:mlp.IN * 64 + 64] = rng.normal(scale=0.1, size=64)  # non-zero biases
    g, loss = pk.pk_costmodel_grad(P, X, t)
    ref_loss, ref_g = mlp.loss_and_grad(P.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss)
    assert np.linalg.norm(g - ref_g) <= 1e-4 * np.linalg.norm(ref_g)
    assert np.max(np.abs(g - ref_g)) <= 1e-4 * np.max(np.abs(ref_g))


@pytest.mark.gpu
def test_adam_step_matches_oracle():
    rng = np.random.default_rng(1)
    f32 = lambda x: x.astype(np.float32).astype(np.float64)  # noqa: E731  the device's inputs, exactly
    P = f32(rng.normal(size=mlp.NPARAM))
    m0 = f32(rng.normal(scale=0.01, size=mlp.NPARAM))
    v0 = f32(np.abs(rng.normal(scale=0.01, size=mlp.NPARAM)))
    g = f32(rng.normal(size=mlp.NPARAM))
    opt = mlp.Adam(mlp.NPARAM, lr=2e-3)
    opt.m, opt.v, opt.t = m0.copy(), v0.copy(), 4          # the device step will be step 5
    ref = opt.step(P.copy(), g)
    Pn, mn, vn = pk.pk_costmodel_adam_step(P, g, m0, v0, 5, 2e-3)
    # float32 arithmetic: each result within a few roundings (u = 2^-24) of
    # the magnitudes that enter it (terms of opposite sign can cancel, so the
    # bound is on the terms, not on the result)
    u = 2.0 ** -24
    b1, b2 = 0.9, 0.999
    assert np.all(np.abs(mn - opt.m) <= 4 * u * (b1 * np.abs(m0) + (1 - b1) * np.abs(g)))
    assert np.all(np.abs(vn - opt.v) <= 5 * u * (b2 * v0 + (1 - b2) * g * g))
    step = np.abs(P - ref)
    assert np.all(np.abs(Pn - ref) <= 4 * u * np.abs(P) + 16 * u * step + 1e-12)


@pytest.mark.gpu
def test_training_fits_a_known_law():
    # time proportional to M N K: ln t = ln M + ln N + ln K + c; the network
    # trained on the device must recover it on unseen shapes
    t = pk.pk_case_table_build(0)
    rng = np.random.default_rng(2)
    dims = np.exp(rng.uniform(np.log(64), np.log(8192), size=(3000, 3)))
    X = np.zeros((3000, mlp.IN), np.float32)
    X[:, :3] = np.log(dims)
    X[:, 3:] = rng.normal(size=(3000, mlp.IN - 3))          # distractors
    secs = np.exp(np.log(dims).sum(1) - 30.0)
    cm, loss = pk.pk_costmodel_train(t, X[:2500], secs[:2500], epochs=1500, lr=3e-3, seed=0)
    assert loss < 1e-2
    pred = cm.predict(X[2500:])
    y = np.log(secs[2500:])
    r2 = 1.0 - np.mean((pred - y) ** 2) / np.var(y)
    assert r2 >= 0.99, r2


@pytest.mark.gpu
def test_shipped_models_pick_programs_that_match_the_oracle():
    # the shipped models (one per element type) attach to a table bound to
    # this device; each LEARNED pick runs and agrees with the oracle
    import torch
    t = pk.pk_case_table_build(0)
    loaded = pk.load_shipped_models(t)
    assert set(loaded) == {"f32", "i32", "bf16"}, loaded
    for dtype, (M, N, K) in (("f32", (1000, 3000, 512)), ("i32", (300, 260, 200)), ("bf16", (512, 384, 264))):
        if dtype == "i32":
            A = inputs.small_int_i32((M, K), seed=5)
            B = inputs.small_int_i32((K, N), seed=6)
        else:
            A = inputs.uniform_f32((M, K), seed=5)
            B = inputs.uniform_f32((K, N), seed=6)
            if dtype == "bf16":
                A, B = inputs.bf16_bits(A), inputs.bf16_bits(B)
        p = pk.pk_select(t, dtype, M, N, K, pk.PK_POLICY_LEARNED)
        C = torch.empty((M, N), dtype=torch.int32 if dtype == "i32" else torch.float32, device="cuda")
        pk.pk_matmul(t, p, dtype, A.cuda(), B.cuda(), C)
        torch.cuda.synchronize()
        ref = om.matmul(A, B, dtype)
        got = C.cpu().numpy()
        if dtype == "i32":
            assert np.array_equal(got, ref), pk.pk_kernel_name(t, p, dtype)
        else:
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            assert err <= (1e-5 if dtype == "f32" else 1e-2), (pk.pk_kernel_name(t, p, dtype), err)
