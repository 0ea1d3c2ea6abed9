"""Host-side tests of libpk.so (no GPU): exported symbols, the symbolic
engine against the oracle and the paper's printed systems, and the bound
matmul case tables against the oracle's brute-force enumerator."""
import json
import os
import re

import numpy as np
import pytest

import oracle.comprehensive as co
import oracle.enumerate as en
from paper_1801_04348_amd import pk
from tests import machines

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "pk.h")) as f:
        text = f.read()
    decls = set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_]+\s*\*?\s*(pk_[a-z_]+)\s*\(", text, re.M))
    assert {"pk_case_table_build", "pk_select", "pk_matmul", "pk_co_solve"} <= decls
    L = pk.lib()
    for name in sorted(decls):
        assert hasattr(L, name), name


def _spec_text(spec):
    """The golden JSON family in the library's text format."""
    sy = spec["symbols"]
    lines = ["machine " + " ".join(sy["machine"]), "program " + " ".join(sy["program"])]
    if sy.get("data"):
        lines.append("data " + " ".join(sy["data"]))
    for s, d in spec["domains"].items():
        if isinstance(d, dict):
            lines.append("domain %s %d %d" % (s, d["lo"], d["hi"]))
        else:
            lines.append("points %s %s" % (s, " ".join(map(str, d))))
    for c in spec["counters"]:
        lines.append("counter %s %s %s" % (c["name"], c["kind"], c["limit"]))
    for c in spec["counters"]:
        for v in c["values"]:
            lines.append("value %s %s : %s" % (c["name"], " ".join(v["when"]), v["value"]))
    for o in spec["strategies"]:
        lines.append("strategy %s %s %s" % (o["name"], "ir" if o["ir"] else "src", " ".join(o["sigma"])))
    if "perf_one" in spec:
        lines.append("perf_one %d" % spec["perf_one"])
    return "\n".join(lines) + "\n"


def _poly(js):
    return co.Poly({tuple(sorted((s, e) for s, e in mono)): c for c, mono in js})


def _lib_leaves(res):
    out = []
    for l in res["leaves"]:
        C = [co.Constraint(_poly(c["lhs"]), _poly(c["rhs"]), c["strict"]) for c in l["system"]]
        out.append((tuple(l["applied"]), tuple(l["lambda"]), C))
    return out


def _same_leaves(lib_leaves, oracle_leaves):
    assert len(lib_leaves) == len(oracle_leaves)
    for (a1, l1, C1), (a2, l2, C2) in zip(lib_leaves, oracle_leaves):
        # compare G_C (source strategies in order) and lambda separately
        assert tuple(a for a in a1 if a not in l1) == tuple(a for a in a2 if a not in l2)
        assert tuple(l1) == tuple(l2)
        assert [c.normal() for c in C1] == [c.normal() for c in C2]


@pytest.mark.parametrize("name", ["fig2_matrix_add", "fig6_jacobi", "fig7_transpose"])
def test_engine_matches_oracle_on_printed_examples(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        spec = json.load(f)
    fam = co.family_from_spec(spec)
    res = pk.pk_co_solve(_spec_text(spec))
    lib_leaves = _lib_leaves(res)
    _same_leaves(lib_leaves, co.solve(fam))
    assert res["height"] == co.tree_height(fam)
    # and directly against the printed systems
    for exp in spec["expected"]:
        want = co.parse_system(exp["system"])
        same = [l for l in lib_leaves if tuple(a for a in l[0] if a not in l[1]) == tuple(exp["variant"])]
        if exp["match"] == "exact":
            assert any(co.equivalent(l[2], want, fam) for l in same), exp
        else:
            assert any(co.implies(want, l[2], fam) for l in same), exp


def test_engine_performance_counter_branch():
    spec = ("machine R P\nprogram b\ndomain R 0 11\ndomain P 0 100\npoints b 1 2\n"
            "counter r resource R\ncounter p performance P\nvalue r : 4*b\nvalue p x : 100\nvalue p : 50\n"
            "strategy x src p\nperf_one 100\n")
    res = pk.pk_co_solve(spec)
    assert len(res["leaves"]) == 1 and res["leaves"][0]["applied"] == []
    texts = [c["text"] for c in res["leaves"][0]["system"]]
    assert "50 <= P" in texts and "4*b <= R" in texts


def test_engine_parse_errors():
    with pytest.raises(pk.PkError) as e:
        pk.pk_co_solve("machine R\ncounter r resource Q\n")
    assert e.value.code == pk.PK_ERR_PARSE


@pytest.fixture(scope="module")
def gfx_table():
    return pk.pk_case_table_build(0, machines.gfx950())


@pytest.fixture(scope="module")
def gfx_desc(gfx_table):
    return pk.pk_case_table_describe(gfx_table)


def test_lds_counter_equals_compiled_lds(gfx_desc):
    for e in gfx_desc["instances"]:
        assert e["lds_bytes"] == e["lds_compiled"], e["name"]
        if e["family"] == en.VALU:
            assert e["lds_bytes"] == en.valu_lds(e["variant"], e["bx"], e["by"], e["s"])
        elif e["family"] == en.VALU2:
            assert e["lds_bytes"] == en.valu2_lds(e["variant"], e["bx"], e["by"], e["s"], e["sy"], e["bk"])
        elif e["family"] == en.TRANSPOSE:
            assert e["lds_bytes"] == en.transpose_lds(e["variant"], e["bx"], e["by"], e["s"])
        elif e["family"] == en.MADD:
            assert e["lds_bytes"] == 0
        elif e["family"] == en.JACOBI:
            assert e["lds_bytes"] == en.jacobi_lds(e["variant"], e["bx"], e["s"])
        elif e["family"] == en.POLYDIV:
            assert e["lds_bytes"] == en.polydiv_lds(e["variant"], e["bx"], e["s"])
        else:
            assert e["lds_bytes"] == en.mfma_lds(e["dtype"], e["variant"], e["bm"], e["bn"], e["bk"])
        # no register spills, except in the float32 single-stage programs of
        # 512 work-items: capped at 128 registers a lane (the 65536-register
        # block budget) while the next K step's loads are in flight, they keep
        # a few loop-invariant values (used only after the unguarded K loop)
        # in scratch across that loop
        if e["family"] == en.MFMA and e["dtype"] == en.F32 and e["threads"] == 512 and e["variant"] == en.SINGLE:
            assert e["scratch"] <= 32, e["name"]
        else:
            assert e["scratch"] == 0, e["name"]


def test_matmul_tables_match_oracle_algorithm(gfx_desc):
    inst = en.InstanceData(gfx_desc["instances"])
    for part in gfx_desc["parts"]:
        fam = en.oracle_family(part["family"], part["dtype"], [tuple(p) for p in part["points"]], inst)
        _same_leaves(_lib_leaves(part["solution"]), co.solve(fam))
        # table symbols: the library's register figures equal the oracle's
        for sym, vals in part["tables"].items():
            got = fam.tables[sym]({s: np.array([p[k] for p in part["points"]])
                                   for k, s in enumerate(fam.program)})
            assert list(got) == vals, sym


def _check_part(part, inst, m):
    """Completeness, soundness and preference of one bound part."""
    fam_id, dt = part["family"], part["dtype"]
    leaves = part["solution"]["leaves"]
    Z, V, T = m.lds_block, m.regs_block, m.max_threads_block
    used = set()
    for i, p in enumerate(part["points"]):
        p = tuple(p)
        some = [v for v in en.variants(fam_id) if en.fits(inst, fam_id, dt, v, p, Z, V, T)]
        leaf = part["first_leaf"][i]
        if some:
            assert leaf >= 0, (fam_id, dt, p, some)                   # completeness
        if leaf >= 0:
            var = leaves[leaf]["variant"]
            assert en.fits(inst, fam_id, dt, var, p, Z, V, T), (p, var)  # soundness
            used.add(leaf)
            if 0 in some:
                assert var == 0, (p, var)                              # preference
    return used


def test_enumerator_over_machine_grid(gfx_desc):
    inst = en.InstanceData(gfx_desc["instances"])
    used = {}
    for Z, V, T in en.machine_grid():
        t = pk.pk_case_table_build(0, machines.grid_machine(Z, V, T))
        d = pk.pk_case_table_describe(t)
        for part in d["parts"]:
            key = (part["family"], part["dtype"])
            used.setdefault(key, set()).update(_check_part(part, inst, machines.grid_machine(Z, V, T)))
    for part in gfx_desc["parts"]:
        n = len(part["solution"]["leaves"])
        key = (part["family"], part["dtype"])
        # no dead leaves: every leaf is selected somewhere on the grid, except
        # register-refusal leaves whose programs never use fewer registers
        dead = [l for l in range(n) if l not in used[key]]
        for l in dead:
            leaf = part["solution"]["leaves"][l]
            assert any("V <" in c["text"] for c in leaf["system"]), leaf


@pytest.mark.parametrize("mk", [machines.gfx950, machines.mi300x_like, machines.fermi_like])
def test_named_machines(mk, gfx_desc):
    inst = en.InstanceData(gfx_desc["instances"])
    m = mk()
    d = pk.pk_case_table_describe(pk.pk_case_table_build(0, m))
    for part in d["parts"]:
        _check_part(part, inst, m)


def test_optimality_definition_3_iv(gfx_desc):
    # for each counter, some leaf at which no strategy of sigma(counter) is
    # left unapplied (so none can lower it further)
    sigma = {0: {"r_Z": {"gran", "nolds"}, "r_V": {"gran", "nolds"}, "r_T": set()},
             1: {"r_Z": {"single"}, "r_V": {"single"}, "r_T": set()},
             2: {"r_Z": {"gran", "nolds"}, "r_V": {"gran", "nolds"}, "r_T": set()},
             3: {"r_V": {"gran"}, "r_T": set()},
             4: {"r_Z": {"gran", "nolds"}, "r_V": {"gran", "nolds"}, "r_T": set()},
             5: {"r_Z": {"gran", "nolds"}, "r_V": {"gran", "nolds"}, "r_T": set()},
             6: {"r_Z": {"gran"}, "r_V": {"gran"}, "r_T": set()}}
    for part in gfx_desc["parts"]:
        for counter, strategies in sigma[part["family"]].items():
            assert any(strategies <= set(l["applied"]) for l in part["solution"]["leaves"]), (part["family"], counter)


def test_height_bound(gfx_desc):
    for part in gfx_desc["parts"]:
        s, t, w = len(part["counters"]), 0, len(part["strategies"])
        assert part["solution"]["height"] <= (s + t) + w * (s + 1)


def test_mi300x_like_drops_to_single_stage():
    # with 64 KiB of LDS the two-stage 256x256 float32 tile (137 KiB) is
    # refused and the one-stage program (69 KiB) still does not fit: no leaf;
    # 128x128 two-stage (69 KiB) is refused, one-stage (34.5 KiB) fits
    t = pk.pk_case_table_build(0, machines.mi300x_like())
    big = pk.params(family=pk.PK_FAMILY_MFMA, bm=256, bn=256, bk=32, wm=4, wn=4)
    with pytest.raises(pk.PkError) as e:
        pk.pk_case_table_lookup(t, "f32", big)
    assert e.value.code == pk.PK_ERR_NO_FEASIBLE_BRANCH
    mid = pk.params(family=pk.PK_FAMILY_MFMA, bm=128, bn=128, bk=32, wm=2, wn=2)
    leaf, var = pk.pk_case_table_lookup(t, "f32", mid)
    assert var == pk.PK_MFMA_SINGLE
    g = pk.pk_case_table_build(0, machines.gfx950())
    assert pk.pk_case_table_lookup(g, "f32", big)[1] == 0


def test_select_returns_feasible_choice(gfx_table):
    for dt in ("f32", "i32", "bf16"):
        for shp in [(1, 1, 1), (256, 256, 256), (1000, 3000, 512), (8192, 8192, 8192)]:
            p = pk.pk_select(gfx_table, dt, *shp)
            leaf, var = pk.pk_case_table_lookup(gfx_table, dt, p)
            assert leaf == p.leaf and var == p.variant


def test_transpose_table_refuses_oversized_workgroups(gfx_table):
    # bx * by = 64 * 32 = 2048 work-items exceeds T = 1024: the refuse branch
    # of r_T has no strategy, so no leaf holds there
    with pytest.raises(pk.PkError) as e:
        pk.pk_case_table_lookup(gfx_table, "f32", pk.params(family=pk.PK_FAMILY_TRANSPOSE, bx=64, by=32, s=1))
    assert e.value.code == pk.PK_ERR_NO_FEASIBLE_BRANCH
    leaf, var = pk.pk_case_table_lookup(gfx_table, "f32", pk.params(family=pk.PK_FAMILY_TRANSPOSE, bx=32, by=8, s=2))
    assert var == 0
    p = pk.pk_select_transpose(gfx_table, "f32", 16384, 16384)
    assert p.family == pk.PK_FAMILY_TRANSPOSE
    # a machine with 4 KiB of LDS: the cached tile of (8 * 8) x 33 words no
    # longer fits, granularity is reduced first, then LDS is dropped
    small = pk.pk_case_table_build(0, machines.variant(lds_block=4096, lds_cu=65536))
    leaf, var = pk.pk_case_table_lookup(small, "f32", pk.params(family=pk.PK_FAMILY_TRANSPOSE, bx=32, by=8, s=8))
    assert var == pk.PK_VALU_GRAN
    leaf, var = pk.pk_case_table_lookup(small, "f32", pk.params(family=pk.PK_FAMILY_TRANSPOSE, bx=64, by=16, s=8))
    assert var == pk.PK_VALU_GRAN | pk.PK_VALU_NOLDS


def test_select_no_feasible_branch():
    t = pk.pk_case_table_build(0, machines.variant(max_threads_block=8))
    with pytest.raises(pk.PkError) as e:
        pk.pk_select(t, "i32", 64, 64, 64)
    assert e.value.code == pk.PK_ERR_NO_FEASIBLE_BRANCH


def test_matmul_argument_errors_without_gpu(gfx_table):
    L = pk.lib()
    rc = L.pk_matmul(gfx_table.handle, None, 0, None, 4, None, 4, None, 4, -1, 4, 4, 0, None)
    assert rc == pk.PK_ERR_INVALID_ARG
    rc = L.pk_matmul(gfx_table.handle, None, 0, 8, 2, 8, 4, 8, 4, 4, 4, 4, 0, None)  # lda < K
    assert rc == pk.PK_ERR_INVALID_ARG
    rc = L.pk_matmul(gfx_table.handle, None, 0, None, 4, None, 4, None, 4, 0, 4, 4, 0, None)  # M == 0
    assert rc == pk.PK_OK
    rc = L.pk_matmul(None, None, 0, None, 4, None, 4, None, 4, 4, 4, 4, 0, None)
    assert rc == pk.PK_ERR_INVALID_ARG
    # the VALU programs have no bfloat16 form
    bad = pk.params(family=pk.PK_FAMILY_VALU, bx=16, by=16, s=1)
    rc = L.pk_matmul(gfx_table.handle, bad, pk.PK_BF16, 16, 4, 16, 4, 16, 4, 4, 4, 4, 0, None)
    assert rc == pk.PK_ERR_UNSUPPORTED_DTYPE


def test_madd_table_has_fig2_shape():
    # Section 1, Fig. 2: two leaves; the unmodified program where its
    # registers fit, else the one-element-per-thread program; both bounded by
    # bx*by <= T.  Machine symbols: V and T only (no LDS in the family).
    d = pk.pk_case_table_describe(pk.pk_case_table_build(0, machines.gfx950()))
    for part in [p for p in d["parts"] if p["family"] == pk.PK_FAMILY_MADD]:
        assert part["counters"] == ["r_V", "r_T"] and part["strategies"] == ["gran"]
        leaves = part["solution"]["leaves"]
        assert [l["applied"] for l in leaves] == [[], ["gran"]]
        texts = [{c["text"] for c in l["system"]} for l in leaves]
        assert {"rho <= V", "bx*by <= T"} <= texts[0]
        assert {"V < rho", "rho_s1 <= V", "bx*by <= T"} <= texts[1]
        assert not any("Z" in t for s in texts for t in s)
        # granularity reduction lowers (or keeps) the register count, as the
        # paper's 14 -> 10 example
        assert all(a >= b for a, b in zip(part["tables"]["rho"], part["tables"]["rho_s1"]))


def test_madd_small_register_file_takes_gran_leaf():
    m = machines.grid_machine(65536, 16384, 1024)
    t = pk.pk_case_table_build(0, m)
    leaf, var = pk.pk_case_table_lookup(t, "f32", pk.params(family=pk.PK_FAMILY_MADD, bx=256, by=4, s=8))
    assert var == pk.PK_VALU_GRAN and leaf == 1        # 40960 registers > V, 16384 after reduction
    leaf, var = pk.pk_case_table_lookup(t, "f32", pk.params(family=pk.PK_FAMILY_MADD, bx=64, by=1, s=8))
    assert var == 0 and leaf == 0
    with pytest.raises(pk.PkError) as e:                # 1024 < bx*by: no leaf
        pk.pk_case_table_lookup(pk.pk_case_table_build(0, machines.grid_machine(65536, 131072, 512)), "i32",
                                pk.params(family=pk.PK_FAMILY_MADD, bx=256, by=4, s=1))
    assert e.value.code == pk.PK_ERR_NO_FEASIBLE_BRANCH
    p = pk.pk_select_madd(t, "i32", 1000, 3000)
    assert p.family == pk.PK_FAMILY_MADD and p.leaf in (0, 1)
    with pytest.raises(pk.PkError):
        pk.pk_select_madd(t, "bf16", 10, 10)


def test_jacobi_table_follows_fig6_cases():
    # Section 5, Fig. 6: the cached program while its LDS fits, granularity 1
    # while that fits, then no LDS; here LDS bytes 4*(s*B + 2) and 4*(B + 2)
    V, T = 131072, 1024
    p = pk.params(family=pk.PK_FAMILY_JACOBI, bx=256, s=8)
    for Z, want in ((65536, 0), (8200, 0), (8199, pk.PK_VALU_GRAN), (1032, pk.PK_VALU_GRAN),
                    (1031, pk.PK_VALU_GRAN | pk.PK_VALU_NOLDS), (0, pk.PK_VALU_GRAN | pk.PK_VALU_NOLDS)):
        t = pk.pk_case_table_build(0, machines.grid_machine(Z, V, T))
        for dt in ("i32", "f32"):
            leaf, var = pk.pk_case_table_lookup(t, dt, p)
            assert var == want, (Z, dt, var)
    d = pk.pk_case_table_describe(pk.pk_case_table_build(0, machines.gfx950()))
    for part in [q for q in d["parts"] if q["family"] == pk.PK_FAMILY_JACOBI]:
        leaves = [(tuple(l["applied"]), {c["text"] for c in l["system"]}) for l in part["solution"]["leaves"]]
        # the three printed cases, each as one leaf (register leaves besides)
        assert any(a == () and "4*B*s + 8 <= Z" in t for a, t in leaves)
        assert any(a == ("gran",) and {"Z < 4*B*s + 8", "4*B + 8 <= Z"} <= t for a, t in leaves)
        assert any(a == ("gran", "nolds") and "Z < 4*B + 8" in t for a, t in leaves)
    t = pk.pk_case_table_build(0, machines.gfx950())
    q = pk.pk_select_jacobi1d(t, "i32", 2 ** 15 + 2)
    assert q.family == pk.PK_FAMILY_JACOBI and q.by == 1
    with pytest.raises(pk.PkError):
        pk.pk_select_jacobi1d(t, "i32", 1)
    with pytest.raises(pk.PkError):
        pk.pk_case_table_lookup(t, "i32", pk.params(family=pk.PK_FAMILY_JACOBI, bx=256, by=2, s=1))


def test_polydiv_table_follows_fig8_cases():
    # Section 5, Fig. 8: the cached program while its LDS fits, granularity 1
    # while that fits, then no LDS; LDS bytes 4*(2*s*B + 1) and 4*(2*B + 1)
    V, T = 131072, 1024
    p = pk.params(family=pk.PK_FAMILY_POLYDIV, bx=128, s=4)
    for Z, want in ((65536, 0), (4100, 0), (4099, pk.PK_VALU_GRAN), (1028, pk.PK_VALU_GRAN),
                    (1027, pk.PK_VALU_GRAN | pk.PK_VALU_NOLDS)):
        t = pk.pk_case_table_build(0, machines.grid_machine(Z, V, T))
        leaf, var = pk.pk_case_table_lookup(t, "i32", p)
        assert var == want, (Z, var)
        with pytest.raises(pk.PkError):
            pk.pk_case_table_lookup(t, "f32", p)
    t = pk.pk_case_table_build(0, machines.gfx950())
    q = pk.pk_select_polydiv(t, 2 ** 15 + 100, 2 ** 15)
    assert q.family == pk.PK_FAMILY_POLYDIV
    with pytest.raises(pk.PkError):
        pk.pk_select_polydiv(t, 10, 0)


def test_polydiv_one_launch_program_selection():
    t = pk.pk_case_table_build(0, machines.gfx950())
    p = pk.pk_select_polydiv(t, 2 ** 15 + 100, 2 ** 15)
    assert p.variant & pk.PK_POLYDIV_FUSED and p.leaf == -1
    assert pk.pk_kernel_name(t, p, "i32").startswith("pk_polydiv_fused_")
    # beyond 1024 quotient coefficients only the per-step programs remain
    p = pk.pk_select_polydiv(t, 5000, 1000)
    assert not (p.variant & pk.PK_POLYDIV_FUSED) and p.leaf >= 0
    # a machine whose LDS cannot hold the quotient falls back to the steps
    small = pk.pk_case_table_build(0, machines.grid_machine(4096, 131072, 1024))
    p = pk.pk_select_polydiv(small, 2 ** 15 + 100, 2 ** 15)
    assert not (p.variant & pk.PK_POLYDIV_FUSED)


def test_case_pick_minimises_the_estimate():
    # pk_select's CASE choice is the feasible (leaf, E) with the least
    # pk_estimate; the feasible set rebuilt from the bound table
    t = pk.pk_case_table_build(0, machines.gfx950())
    d = pk.pk_case_table_describe(t)
    ncu = d["machine"]["cu_count"]
    for dtype, dt in (("f32", 0), ("i32", 1), ("bf16", 2)):
        for M, N, K in ((512, 512, 512), (3000, 8192, 1000), (100, 2000, 64), (512, 512, 8192)):
            cands = []
            for part in d["parts"]:
                fam = part["family"]
                if part["dtype"] != dt or fam not in (pk.PK_FAMILY_VALU, pk.PK_FAMILY_VALU2, pk.PK_FAMILY_MFMA):
                    continue
                for i, pt in enumerate(part["points"]):
                    if part["first_leaf"][i] < 0:
                        continue
                    if fam == pk.PK_FAMILY_VALU:
                        cands.append(pk.params(family=fam, bx=pt[0], by=pt[1], s=pt[2]))
                    elif fam == pk.PK_FAMILY_VALU2:
                        cands.append(pk.params(family=fam, bx=pt[0], by=pt[1], s=pt[2], sy=pt[3], bk=pt[4]))
                    else:
                        cands.append(pk.params(family=fam, bm=pt[0], bn=pt[1], bk=pt[2], wm=pt[3], wn=pt[4]))
                        # the shares of K offered: fewer tiles than two per
                        # compute unit at the previous count, two K steps a share
                        # (programs with a split form: the library refuses the others)
                        tiles = -(-M // pt[0]) * -(-N // pt[1])
                        ks = 2
                        while ks <= 16 and 2 * ks <= -(-K // pt[2]) and tiles * (ks // 2) < 2 * ncu:
                            q = pk.params(family=fam, bm=pt[0], bn=pt[1], bk=pt[2], wm=pt[3], wn=pt[4], ks=ks)
                            try:
                                pk.pk_kernel_name(t, q, dtype)
                            except pk.PkError:
                                break
                            cands.append(q)
                            ks *= 2
            est = [pk.pk_estimate(t, p, dtype, M, N, K) for p in cands]
            assert all(e > 0 for e in est)
            best = cands[min(range(len(est)), key=est.__getitem__)]
            pick = pk.pk_select(t, dtype, M, N, K, pk.PK_POLICY_CASE)
            assert (pk.pk_kernel_name(t, pick, dtype), pick.ks) == (pk.pk_kernel_name(t, best, dtype), best.ks), \
                (dtype, M, N, K)
    with pytest.raises(pk.PkError):
        pk.pk_estimate(t, pk.params(family=pk.PK_FAMILY_TRANSPOSE, bx=32, by=8, s=1), "f32", 1, 1, 1)


def test_every_mfma_program_has_an_element_load_twin(gfx_desc):
    # the twin reads unaligned rows; the program's register symbol covers both
    inst = {e["name"]: e for e in gfx_desc["instances"]}
    single = [e for e in gfx_desc["instances"]
              if e["family"] == en.MFMA and not e["variant"] & (2 | en.ELEMENT | pk.PK_MFMA_SPLIT)]
    for e in single:
        twin = inst.get(e["name"] + "_el")
        # bf16 tiles built without a twin (it would spill): the largest, and
        # those of K tile 64 on four wavefronts with 128 x 256 outputs
        if e["dtype"] == 2 and (e["bm"] * e["bn"] >= 256 * 256 or
                                (e["bk"] == 64 and e["wm"] * e["wn"] == 4 and e["bm"] * e["bn"] >= 128 * 256)):
            assert twin is None
            continue
        assert twin is not None and twin["variant"] == e["variant"] | en.ELEMENT, e["name"]
        assert twin["lds_bytes"] == e["lds_bytes"] and twin["scratch"] == 0
        # the split form (shares of K) of a wide program up to 512 work-items
        split = inst.get(e["name"] + "_sk")
        if split is not None:
            assert e["threads"] <= 512 and split["variant"] == e["variant"] | pk.PK_MFMA_SPLIT
            assert split["lds_bytes"] == e["lds_bytes"] and split["scratch"] == 0
    assert sum(1 for e in gfx_desc["instances"] if e["variant"] & pk.PK_MFMA_SPLIT) > 0
    data = en.InstanceData(gfx_desc["instances"])
    for part in gfx_desc["parts"]:
        if part["family"] != en.MFMA:
            continue
        for sym, vals in part["tables"].items():
            v = en.SINGLE if "one" in sym else 0
            for pt, val in zip(part["points"], vals):
                e = inst["pk_mfma_%s_%dx%dx%d_w%dx%d_st%d" % ({0: "f32", 1: "i32", 2: "bf16"}[part["dtype"]], *pt,
                                                             1 if v else 2)]
                own = en.regs_per_block(e["vgpr"], e["agpr"], e["threads"])
                assert val == data.regs(en.MFMA, part["dtype"], v, tuple(pt)) and val >= own
