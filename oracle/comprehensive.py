"""Comprehensive optimization (Section 3) -- TEST INFRASTRUCTURE ONLY.

A plain transcription of the method's steps in the paper's notation:

* a code fragment S is described by a ``Family``: its machine parameters
  (resource limits R_i and performance measures P_i), program parameters E_j,
  data parameters D_k, its resource counters r_i and performance counters p_i
  (each evaluated on the fragment after a given set of optimization strategies,
  Section 3.3), and its optimization strategies O_1..O_w with the sets
  sigma(r_i), sigma(p_i) of counters each may improve (Section 3.4);
* the quintuple Q(S) = (G_C, lambda, omega, gamma, C) of Section 3.6, with the
  stack conventions of Remark 2 (pop takes the head; pushing t_1..t_M puts
  t_M first);
* Algorithm 1 (ComprehensiveOptimization) and Algorithm 2 (Optimize), with
  the accept branch (0 <= v <= R) and the refuse branch (R < v, then the first
  strategy of sigma(c) still in omega) for resource counters, and
  (0 <= v <= P) / (P < v <= 1) for performance counters.

Consistency of a constraint system (Definition 3 (i)) is decided here by
brute force over finite integer domains given for every symbol (parameters
are non-negative integers by hypothesis H1), not over the reals.  Machine
symbols that occur in separate constraints are enumerated separately (a
conjunction of constraints on disjoint symbol sets is satisfiable iff each
part is), everything else jointly, so the check stays exact.

Polynomials have integer coefficients.  A *table symbol* stands for a number
that depends on the program parameters through a lookup (e.g. the registers
a compiled instance uses); it is evaluated from the program-parameter grid.
"""
from __future__ import annotations

import copy
import itertools
import re
from dataclasses import dataclass, field
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# polynomials with integer coefficients


class Poly:
    """Sparse polynomial: {monomial: coefficient}, monomial = sorted tuple of
    (symbol, exponent) pairs; the empty tuple is the constant term."""

    __slots__ = ("terms",)

    def __init__(self, terms: Optional[Dict[tuple, int]] = None):
        self.terms = {m: c for m, c in (terms or {}).items() if c != 0}

    @staticmethod
    def const(c: int) -> "Poly":
        return Poly({(): int(c)})

    @staticmethod
    def sym(name: str) -> "Poly":
        return Poly({((name, 1),): 1})

    def __add__(self, o):
        o = _as_poly(o)
        t = dict(self.terms)
        for m, c in o.terms.items():
            t[m] = t.get(m, 0) + c
        return Poly(t)

    __radd__ = __add__

    def __neg__(self):
        return Poly({m: -c for m, c in self.terms.items()})

    def __sub__(self, o):
        return self + (-_as_poly(o))

    def __rsub__(self, o):
        return _as_poly(o) - self

    def __mul__(self, o):
        o = _as_poly(o)
        t: Dict[tuple, int] = {}
        for m1, c1 in self.terms.items():
            for m2, c2 in o.terms.items():
                d: Dict[str, int] = {}
                for s, e in m1 + m2:
                    d[s] = d.get(s, 0) + e
                m = tuple(sorted(d.items()))
                t[m] = t.get(m, 0) + c1 * c2
        return Poly(t)

    __rmul__ = __mul__

    def __pow__(self, e: int):
        r = Poly.const(1)
        for _ in range(e):
            r = r * self
        return r

    def __eq__(self, o):
        return isinstance(o, Poly) and self.terms == o.terms

    def __hash__(self):
        return hash(self.key())

    def key(self):
        return tuple(sorted(self.terms.items()))

    def symbols(self) -> set:
        return {s for m in self.terms for s, _ in m}

    def is_const(self) -> bool:
        return all(m == () for m in self.terms)

    def const_value(self) -> int:
        return self.terms.get((), 0)

    def evaluate(self, env: Dict[str, object]):
        total = 0
        for m, c in self.terms.items():
            v = c
            for s, e in m:
                v = v * (env[s] ** e)
            total = total + v
        return total

    def __repr__(self):
        if not self.terms:
            return "0"
        parts = []
        for m, c in sorted(self.terms.items(), key=lambda mc: (-len(mc[0]), mc[0])):
            mono = "*".join(s if e == 1 else "%s^%d" % (s, e) for s, e in m)
            if not mono:
                parts.append(str(c))
            elif c == 1:
                parts.append(mono)
            elif c == -1:
                parts.append("-" + mono)
            else:
                parts.append("%d*%s" % (c, mono))
        return " + ".join(parts).replace("+ -", "- ")


def _as_poly(x) -> Poly:
    if isinstance(x, Poly):
        return x
    if isinstance(x, (int, np.integer)):
        return Poly.const(int(x))
    if isinstance(x, str):
        return parse_poly(x)
    raise TypeError("cannot make a polynomial of %r" % (x,))


_TOK = re.compile(r"\s*(?:(\d+)|([A-Za-z_][A-Za-z_0-9]*)|(<=|<|\+|-|\*|\^|\(|\)))")


def _tokens(text: str) -> List[str]:
    pos, out = 0, []
    text = text.strip()
    while pos < len(text):
        m = _TOK.match(text, pos)
        if not m or m.end() == pos:
            raise ValueError("cannot parse %r at %d" % (text, pos))
        out.append(m.group(1) or m.group(2) or m.group(3))
        pos = m.end()
    return out


def parse_poly(text: str) -> Poly:
    toks = _tokens(text)
    p, i = _parse_expr(toks, 0)
    if i != len(toks):
        raise ValueError("trailing input in %r" % text)
    return p


def _parse_expr(t, i):
    p, i = _parse_term(t, i)
    while i < len(t) and t[i] in "+-":
        op = t[i]
        q, i = _parse_term(t, i + 1)
        p = p + q if op == "+" else p - q
    return p, i


def _parse_term(t, i):
    p, i = _parse_factor(t, i)
    while i < len(t) and t[i] == "*":
        q, i = _parse_factor(t, i + 1)
        p = p * q
    return p, i


def _parse_factor(t, i):
    if t[i] == "-":
        p, i = _parse_factor(t, i + 1)
        return -p, i
    if t[i] == "(":
        p, i = _parse_expr(t, i + 1)
        if t[i] != ")":
            raise ValueError("missing )")
        i += 1
    elif t[i].isdigit():
        p, i = Poly.const(int(t[i])), i + 1
    else:
        p, i = Poly.sym(t[i]), i + 1
    if i < len(t) and t[i] == "^":
        p, i = p ** int(t[i + 1]), i + 2
    return p, i


# ---------------------------------------------------------------------------
# constraints


@dataclass(frozen=True)
class Constraint:
    """lhs <= rhs (strict=False) or lhs < rhs (strict=True)."""

    lhs: Poly
    rhs: Poly
    strict: bool

    def holds(self, env):
        a, b = self.lhs.evaluate(env), self.rhs.evaluate(env)
        return (a < b) if self.strict else (a <= b)

    def symbols(self) -> set:
        return self.lhs.symbols() | self.rhs.symbols()

    def normal(self):
        """(difference lhs - rhs, strict): the canonical form used to compare."""
        return ((self.lhs - self.rhs).key(), self.strict)

    def __repr__(self):
        return "%r %s %r" % (self.lhs, "<" if self.strict else "<=", self.rhs)


def le(a, b) -> Constraint:
    return Constraint(_as_poly(a), _as_poly(b), False)


def lt(a, b) -> Constraint:
    return Constraint(_as_poly(a), _as_poly(b), True)


def parse_system(lines: Iterable[str]) -> List[Constraint]:
    """Parse constraints such as ``"10 <= R < 14"`` (chains split in two)."""
    out = []
    for line in lines:
        parts = re.split(r"(<=|<)", line)
        if len(parts) < 3:
            raise ValueError("not a constraint: %r" % line)
        exprs = [parse_poly(p) for p in parts[0::2]]
        rels = parts[1::2]
        for k, r in enumerate(rels):
            out.append(Constraint(exprs[k], exprs[k + 1], r == "<"))
    return out


# ---------------------------------------------------------------------------
# the code fragment description


@dataclass
class Counter:
    name: str
    kind: str            # "resource" or "performance"
    limit: str           # the machine symbol R_i or P_i it is compared with
    value: Callable[[Tuple[str, ...]], Poly]   # evaluation on S after strategies


@dataclass
class Strategy:
    name: str
    on_ir: bool          # applied to the IR (recorded in lambda) or to the source
    sigma: frozenset     # names of the counters it may improve


@dataclass
class Family:
    machine: List[str]
    program: List[str]
    data: List[str]
    counters: List[Counter]            # r_1..r_s then p_1..p_t, in gamma order
    strategies: List[Strategy]         # O_1..O_w, in omega order
    domains: Dict[str, Sequence[int]]  # finite integer domain of every symbol
    tables: Dict[str, Callable[[Dict[str, np.ndarray]], np.ndarray]] = field(default_factory=dict)
    # the value that stands for 1 (100 %) in the units performance measures
    # and counters are given in, so that they stay integers
    perf_one: int = 1
    # when given, the (program, data) parameter values range over this list
    # of tuples (in the order program + data) instead of the product of the
    # per-symbol domains
    points: Optional[List[Tuple[int, ...]]] = None

    # performance measures are the machine symbols limiting performance counters
    def perf_symbols(self):
        return {c.limit for c in self.counters if c.kind == "performance"}


# ---------------------------------------------------------------------------
# consistency by brute force over finite domains (Definition 3 (i); integer
# points per hypothesis H1)


def consistent(system: Sequence[Constraint], fam: Family) -> bool:
    syms = set()
    for c in system:
        syms |= c.symbols()
    machine = [s for s in fam.machine if s in syms]
    table_syms = [s for s in fam.tables if s in syms]
    grid_syms = [s for s in list(fam.program) + list(fam.data) if s in syms]
    if table_syms:  # tables depend on every program parameter
        grid_syms = [s for s in list(fam.program) + list(fam.data)]
    grid_syms = sorted(set(grid_syms), key=lambda s: (list(fam.program) + list(fam.data)).index(s))
    unknown = syms - set(machine) - set(table_syms) - set(grid_syms)
    if unknown:
        raise ValueError("symbols without a domain: %s" % sorted(unknown))

    # joint grid over program/data parameters
    if fam.points is not None:
        order = list(fam.program) + list(fam.data)
        arr = np.asarray(fam.points, dtype=np.int64).reshape(len(fam.points), len(order))
        env = {s: arr[:, k] for k, s in enumerate(order)}
        npts = arr.shape[0]
    elif grid_syms:
        axes = np.meshgrid(*[np.asarray(fam.domains[s], dtype=np.int64) for s in grid_syms], indexing="ij")
        env = {s: a.reshape(-1) for s, a in zip(grid_syms, axes)}
        npts = env[grid_syms[0]].size
    else:
        env, npts = {}, 1
    for t in table_syms:
        env[t] = np.asarray(fam.tables[t](env), dtype=np.int64).reshape(-1)

    # group constraints by the machine symbols they mention (union-find)
    parent = {m: m for m in machine}

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x

    for c in system:
        ms = [m for m in machine if m in c.symbols()]
        for a, b in zip(ms, ms[1:]):
            parent[find(a)] = find(b)
    groups: Dict[Optional[str], List[Constraint]] = {}
    for c in system:
        ms = [m for m in machine if m in c.symbols()]
        key = find(ms[0]) if ms else None
        groups.setdefault(key, []).append(c)

    ok = np.ones(npts, dtype=bool)
    for key, cons in groups.items():
        if key is None:
            for c in cons:
                ok &= np.broadcast_to(np.asarray(c.holds(env)), (npts,))
            continue
        members = [m for m in machine if find(m) == key]
        maxes = np.meshgrid(*[np.asarray(fam.domains[m], dtype=np.int64) for m in members], indexing="ij")
        mvals = {m: a.reshape(-1) for m, a in zip(members, maxes)}
        nm = mvals[members[0]].size
        full = {s: v[:, None] for s, v in env.items()}
        full.update({m: v[None, :] for m, v in mvals.items()})
        sat = np.ones((npts, nm), dtype=bool)
        for c in cons:
            sat &= np.broadcast_to(np.asarray(c.holds(full)), (npts, nm))
        ok &= sat.any(axis=1)
    return bool(ok.any())


# ---------------------------------------------------------------------------
# quintuple and the two algorithms


@dataclass
class Quintuple:
    GC: Tuple[str, ...]          # source-level strategies applied to S (identifies G_C)
    lam: List[str]               # lambda: strategies applied to the IR
    omega: List[str]             # strategies not applied yet
    gamma: List[str]             # counters still to evaluate (head = next)
    C: List[Constraint]          # constraints computed so far

    def applied(self) -> Tuple[str, ...]:
        return tuple(self.GC) + tuple(self.lam)


def _push(stack: list, item):
    """Remark 2 (2): pushing t onto s_1..s_N gives t, s_1..s_N."""
    stack.insert(0, item)


def _push_seq(stack: list, items: Sequence):
    """Remark 2 (3): pushing t_1..t_M gives t_M..t_1, s_1..s_N."""
    for t in items:
        stack.insert(0, t)


def initial_quintuple(fam: Family) -> Quintuple:
    """Q(S) at the start: lambda empty, omega = O_1..O_w, gamma = r_1..r_s,
    p_1..p_t, C = non-negativity of every parameter and 0 <= P_i <= 1."""
    C = []
    perf = fam.perf_symbols()
    for s in fam.machine:
        C.append(le(0, s))
        if s in perf:
            C.append(le(s, fam.perf_one))
    for s in list(fam.data) + list(fam.program):
        C.append(le(0, s))
    return Quintuple(GC=(), lam=[], omega=[o.name for o in fam.strategies],
                     gamma=[c.name for c in fam.counters], C=C)


def optimize(Q: Quintuple, fam: Family) -> List[Quintuple]:
    """Algorithm 2."""
    counters = {c.name: c for c in fam.counters}
    strategies = {o.name: o for o in fam.strategies}
    resources = [c.name for c in fam.counters if c.kind == "resource"]
    result: List[Quintuple] = []
    cname = Q.gamma.pop(0)                     # take the next counter out of gamma
    c = counters[cname]
    v = c.value(Q.applied())                   # evaluate it on S'
    Q2 = copy.deepcopy(Q)                      # the refuse branch starts as a copy
    if c.kind == "resource":
        Q.C += [le(0, v), le(v, c.limit)]      # accept: 0 <= v <= R_i
        _push(result, Q)
        Q2.C.append(lt(c.limit, v))            # refuse: R_i < v
        pushed = resources[: resources.index(cname) + 1]          # r_1..r_i
    else:
        Q.C += [le(0, v), le(v, c.limit)]      # accept: 0 <= v <= P_i
        _push(result, Q)
        Q2.C += [lt(c.limit, v), le(v, fam.perf_one)]   # refuse: P_i < v <= 1
        pushed = resources + [cname]                              # r_1..r_s, p_i
    chosen = next((o for o in Q2.omega if cname in strategies[o].sigma), None)
    if chosen is None:
        return result
    Q3 = Q2                                    # apply the strategy to S''
    Q3.omega = [o for o in Q3.omega if o != chosen]
    if strategies[chosen].on_ir:
        Q3.lam = Q3.lam + [chosen]
    else:
        Q3.GC = tuple(Q3.GC) + (chosen,)
    _push_seq(Q3.gamma, pushed)
    _push_seq(result, optimize(Q3, fam))
    return [q for q in result if consistent(q.C, fam)]


def comprehensive_optimization(Q: Quintuple, fam: Family):
    """Algorithm 1.  Returns the output stack of ((G_C, lambda), C) pairs.

    A processed quintuple whose system is inconsistent is not returned: the
    paper maintains every system through RealTriangularize, which detects
    inconsistency as constraints are added (Section 3.7, remarks R5 and R6),
    so no output system is empty (Definition 3 (i))."""
    if not Q.gamma:
        if not consistent(Q.C, fam):
            return []
        return [((tuple(Q.GC), tuple(Q.lam)), list(Q.C))]
    out: list = []
    for Qp in optimize(Q, fam):
        _push_seq(out, comprehensive_optimization(Qp, fam))
    return out


def solve(fam: Family):
    """Run Algorithm 1 from the initial quintuple; returns a list of leaves
    (applied strategies in order, lambda, constraint list)."""
    leaves = comprehensive_optimization(initial_quintuple(fam), fam)
    return [(gc + lam, lam, C) for (gc, lam), C in leaves]


def tree_height(fam: Family) -> int:
    """Height of the tree T(Q(S)) of Section 3.7: every evaluation of a
    counter is a node with an accept edge and, when a strategy of sigma(c) is
    left in omega, a refuse edge (T2.1, T2.2).  Lemma 1 bounds it by w(s+t)."""
    counters = {c.name: c for c in fam.counters}
    strategies = {o.name: o for o in fam.strategies}
    resources = [c.name for c in fam.counters if c.kind == "resource"]

    def height(Q: Quintuple) -> int:
        if not Q.gamma:
            return 0
        cname = Q.gamma.pop(0)
        c = counters[cname]
        v = c.value(Q.applied())
        acc = copy.deepcopy(Q)
        acc.C += [le(0, v), le(v, c.limit)]
        h = 1 + height(acc)
        ref = copy.deepcopy(Q)
        if c.kind == "resource":
            ref.C.append(lt(c.limit, v))
            pushed = resources[: resources.index(cname) + 1]
        else:
            ref.C += [lt(c.limit, v), le(v, fam.perf_one)]
            pushed = resources + [cname]
        chosen = next((o for o in ref.omega if cname in strategies[o].sigma), None)
        if chosen is None:
            return h
        ref.omega = [o for o in ref.omega if o != chosen]
        if strategies[chosen].on_ir:
            ref.lam = ref.lam + [chosen]
        else:
            ref.GC = tuple(ref.GC) + (chosen,)
        _push_seq(ref.gamma, pushed)
        return max(h, 1 + height(ref))

    return height(initial_quintuple(fam))


# ---------------------------------------------------------------------------
# comparing systems


def drop_trivial(system: Sequence[Constraint], fam: Family) -> List[Constraint]:
    """Remove constraints that hold at every point of the domains and
    duplicates; what is left is compared with the printed systems."""
    out, seen = [], set()
    for c in system:
        k = c.normal()
        if k in seen:
            continue
        seen.add(k)
        if _always(c, fam):
            continue
        out.append(c)
    return out


def _always(c: Constraint, fam: Family) -> bool:
    neg = Constraint(c.rhs, c.lhs, not c.strict)   # not(a <= b) is b < a
    return not consistent([neg], fam)


def equivalent(s1: Sequence[Constraint], s2: Sequence[Constraint], fam: Family) -> bool:
    """Same solution set over the finite domains: s1 implies every constraint
    of s2 and conversely."""
    for a, b in ((s1, s2), (s2, s1)):
        for c in b:
            neg = Constraint(c.rhs, c.lhs, not c.strict)
            if consistent(list(a) + [neg], fam):
                return False
    return True


def implies(s1: Sequence[Constraint], s2: Sequence[Constraint], fam: Family) -> bool:
    """Every solution of s1 is a solution of s2."""
    for c in s2:
        neg = Constraint(c.rhs, c.lhs, not c.strict)
        if consistent(list(s1) + [neg], fam):
            return False
    return True


def family_from_spec(spec: dict) -> Family:
    """Build a Family from a JSON-like description in which each counter gives
    its value as a list of (strategies that must have been applied, polynomial)
    entries; the first entry whose strategies are all applied is the value."""
    counters = []
    for c in spec["counters"]:
        entries = [(frozenset(e["when"]), parse_poly(e["value"])) for e in c["values"]]

        def value(applied, entries=entries, name=c["name"]):
            a = set(applied)
            for when, poly in entries:
                if when <= a:
                    return poly
            raise ValueError("no value of %s after %s" % (name, applied))

        counters.append(Counter(c["name"], c["kind"], c["limit"], value))
    strategies = [Strategy(o["name"], bool(o["ir"]), frozenset(o["sigma"])) for o in spec["strategies"]]
    doms = {}
    for s, d in spec["domains"].items():
        if isinstance(d, dict):
            doms[s] = list(range(d["lo"], d["hi"] + 1))
        else:
            doms[s] = list(d)
    sy = spec["symbols"]
    return Family(machine=list(sy["machine"]), program=list(sy["program"]), data=list(sy.get("data", [])),
                  counters=counters, strategies=strategies, domains=doms, perf_one=int(spec.get("perf_one", 1)))
