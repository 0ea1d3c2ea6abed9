"""Pins of the comprehensive-optimization oracle (Algorithms 1 and 2).

What fixes the expected values: the constraint systems the paper prints for
its worked examples (Fig. 2, Fig. 6, Fig. 7; fixtures under tests/golden/ with
their citations), the stack conventions of Remark 2, coverage (Definition 3
(iii)) checked by brute force, and hand-worked small families.
"""
import json
import os

import numpy as np
import pytest

import oracle.comprehensive as co

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        spec = json.load(f)
    return spec, co.family_from_spec(spec)


def _gc(leaf):
    applied, lam, C = leaf
    return tuple(a for a in applied if a not in lam)


@pytest.mark.parametrize("name", ["fig2_matrix_add", "fig6_jacobi"])
def test_printed_systems_reproduced_exactly(name):
    spec, fam = _load(name)
    leaves = co.solve(fam)
    assert len(leaves) == len(spec["expected"])
    unmatched = list(leaves)
    for exp in spec["expected"]:
        want = co.parse_system(exp["system"])
        hit = [l for l in unmatched if _gc(l) == tuple(exp["variant"]) and co.equivalent(l[2], want, fam)]
        assert len(hit) == 1, (exp, [(_gc(l), co.drop_trivial(l[2], fam)) for l in leaves])
        unmatched.remove(hit[0])
    assert not unmatched


def test_fig2_structural_match():
    # beyond equivalence: after dropping always-true and duplicate
    # constraints the systems are literally the printed ones
    spec, fam = _load("fig2_matrix_add")
    got = {(_gc(l), frozenset(c.normal() for c in co.drop_trivial(l[2], fam))) for l in co.solve(fam)}
    want = {(tuple(e["variant"]), frozenset(c.normal() for c in co.parse_system(e["system"])))
            for e in spec["expected"]}
    assert got == want


def test_fig7_printed_systems():
    spec, fam = _load("fig7_transpose")
    leaves = co.solve(fam)
    for exp in spec["expected"]:
        want = co.parse_system(exp["system"])
        same = [l for l in leaves if _gc(l) == tuple(exp["variant"])]
        if exp["match"] == "exact":
            assert any(co.equivalent(l[2], want, fam) for l in same), exp
        else:
            assert any(co.implies(want, l[2], fam) for l in same), exp
    # the leaf the printed list lacks: registers refused at 6, granularity reduced
    extra = co.parse_system(["2*s*B0*B1 <= Z_B", "5 <= R_B < 6"])
    assert any(_gc(l) == ("gran",) and co.equivalent(l[2], extra, fam) for l in leaves)
    assert len(leaves) == 4


def _fits(fam, variant, env):
    """Does the fragment after the strategies in ``variant`` fit the machine
    at point ``env`` (every resource counter within its limit)?"""
    ok = np.ones_like(next(iter(env.values())), dtype=bool)
    for c in fam.counters:
        if c.kind != "resource":
            continue
        ok &= np.asarray(co.le(c.value(variant), c.limit).holds(env))
    return ok


def _grid(fam):
    syms = list(fam.machine) + list(fam.program) + list(fam.data)
    axes = np.meshgrid(*[np.asarray(fam.domains[s]) for s in syms], indexing="ij")
    return {s: a.reshape(-1) for s, a in zip(syms, axes)}


@pytest.mark.parametrize("name", ["fig2_matrix_add", "fig6_jacobi", "fig7_transpose"])
def test_coverage_definition_3_iii(name):
    # wherever some program the strategies can produce fits the machine, some
    # leaf's system holds (every refuse carries the negation of its accept)
    spec, fam = _load(name)
    env = _grid(fam)
    variants = {()}
    for o in fam.strategies:
        variants |= {v + (o.name,) for v in variants}
    some_fits = np.zeros(env[fam.machine[0]].size, dtype=bool)
    for v in variants:
        some_fits |= _fits(fam, v, env)
    covered = np.zeros_like(some_fits)
    for leaf in co.solve(fam):
        held = np.ones_like(covered)
        for c in leaf[2]:
            held &= np.asarray(c.holds(env))
        covered |= held
        # soundness: where a leaf holds, its own program fits
        assert np.all(_fits(fam, leaf[0], env)[held])
    assert np.all(covered[some_fits])


def test_fig7_printed_list_lacks_coverage():
    # why the reading of Fig. 7 keeps the algorithm's extra leaf: at R_B = 5
    # and Z_B >= 2 s B0 B1 the reduced-granularity program fits but no printed
    # system holds
    spec, fam = _load("fig7_transpose")
    env = {"R_B": 5, "Z_B": 64, "s": 2, "B0": 4, "B1": 4}
    assert _fits(fam, ("gran",), {k: np.array([v]) for k, v in env.items()})[0]
    for exp in spec["expected"]:
        assert not all(c.holds(env) for c in co.parse_system(exp["system"]))


def test_remark2_stack_conventions():
    s = ["s1", "s2"]
    co._push(s, "t")
    assert s == ["t", "s1", "s2"]
    s = ["s1", "s2"]
    co._push_seq(s, ["t1", "t2", "t3"])
    assert s == ["t3", "t2", "t1", "s1", "s2"]


def test_refuse_repushes_counters_in_remark2_order():
    # Fig. 7 family, r_Z already accepted at 2sB0B1, r_R (6) next.  Refusing
    # R_B < 6 applies regpressure (an IR strategy, so it goes to lambda) and
    # pushes r_1, r_2 = r_Z, r_R, i.e. gamma = (r_R, r_Z): r_R is evaluated
    # again first (still 6, accept inconsistent), is refused again, and
    # granularity is reduced, pushing r_Z, r_R once more.  The surviving
    # accept (5 <= R_B) therefore still has r_Z twice in gamma.
    spec, fam = _load("fig7_transpose")
    Q = co.initial_quintuple(fam)
    Q.gamma = ["r_R"]
    Q.C += co.parse_system(["2*s*B0*B1 <= Z_B"])
    out = co.optimize(Q, fam)
    states = sorted((q.GC, tuple(q.lam), tuple(q.gamma)) for q in out)
    assert states == [((), (), ()), (("gran",), ("regpressure",), ("r_Z", "r_Z"))]


def test_lemma1_height():
    # Lemma 1 argues at most w refuse edges and runs of at most s+t accept
    # edges.  Refuse branches re-push r_1..r_i (or r_1..r_s, p_i), so a run of
    # accepts can be longer than s+t: the literal algorithm's height is
    # bounded by (s+t) + w*(s+1) instead; termination still holds.
    for name in ("fig2_matrix_add", "fig6_jacobi", "fig7_transpose"):
        spec, fam = _load(name)
        w = len(fam.strategies)
        s = sum(c.kind == "resource" for c in fam.counters)
        t = len(fam.counters) - s
        assert co.tree_height(fam) <= (s + t) + w * (s + 1)
    spec, fam = _load("fig6_jacobi")
    assert co.tree_height(fam) == 7 > 3 * 2   # exceeds the printed w(s+t)


def test_consistency_brute_force_cases():
    fam = co.Family(machine=["R", "Z"], program=["b"], data=[], counters=[], strategies=[],
                    domains={"R": range(0, 20), "Z": range(0, 20), "b": [1, 2, 3]})
    P = co.parse_system
    assert not co.consistent(P(["R < 10", "10 <= R"]), fam)
    assert co.consistent(P(["9 <= R < 10"]), fam)
    assert not co.consistent(P(["Z + R <= 3", "2 <= Z", "2 <= R"]), fam)      # joint symbols
    assert co.consistent(P(["Z + R <= 4", "2 <= Z", "2 <= R"]), fam)
    assert not co.consistent(P(["4*b <= R", "R < 4", "0 <= b"]), fam)         # b >= 1 in its domain
    assert co.consistent(P(["4*b <= R", "R < 5"]), fam)
    assert not co.consistent(P(["3*b <= Z", "Z < 3*b"]), fam)


def test_performance_counter_branch_literal():
    # A hand-worked family with one resource counter r (value 4b, limit R)
    # and one performance counter p (occupancy in percent: 50, or 100 after
    # strategy x).  Algorithm 2 accepts p with 0 <= 50 <= P and refuses with
    # P < 50 <= 100; applying x raises p to 100, whose accept 100 <= P
    # contradicts P < 50 -- the branch is discarded, as remark R3 says
    # happens when a strategy makes the estimate larger.
    fam = co.Family(
        machine=["R", "P"], program=["b"], data=[],
        counters=[co.Counter("r", "resource", "R", lambda a: co.parse_poly("4*b")),
                  co.Counter("p", "performance", "P", lambda a: co.Poly.const(100 if "x" in a else 50))],
        strategies=[co.Strategy("x", False, frozenset({"p"}))],
        domains={"R": range(0, 12), "P": range(0, 101), "b": [1, 2]}, perf_one=100)
    leaves = co.solve(fam)
    assert len(leaves) == 1
    assert leaves[0][0] == ()
    assert co.equivalent(leaves[0][2], co.parse_system(["4*b <= R", "50 <= P"]), fam)
    # a strategy that leaves the estimate unchanged keeps the refuse branch
    fam.counters[1] = co.Counter("p", "performance", "P", lambda a: co.Poly.const(50))
    leaves = co.solve(fam)
    got = sorted((l[0], tuple(sorted(map(repr, co.drop_trivial(l[2], fam))))) for l in leaves)
    assert len(leaves) == 1 and leaves[0][0] == ()


def test_polynomial_parser_and_arithmetic():
    p = co.parse_poly("2*s*B + 2")
    assert p.evaluate({"s": 3, "B": 5}) == 32
    q = co.parse_poly("(B0 + 1)^2 - B0*B0 - 2*B0")
    assert q.is_const() and q.const_value() == 1
    assert co.parse_poly("-3*x + x*2").evaluate({"x": 7}) == -7
