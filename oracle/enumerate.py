"""Brute-force enumerator of the matmul families' resource constraints --
TEST INFRASTRUCTURE ONLY.

Re-derives, from the kernels' documented layouts, what every program of the
two matmul families needs, and checks a bound case table against it by
enumeration over a grid of machines and the whole program-parameter domain:

* VALU family (the blocked kernel of Section 2, Fig. 4): program parameters
  bx, by, s, K tile bk = by; programs ("variants") are the strategy sets
  {} (LDS-tiled, s outputs per thread), {gran} (LDS-tiled, 1 output per
  thread), {gran, nolds} and {nolds} (no LDS).  LDS bytes of a tiled program:
  4 * (by * (bk + 1) + bk * bx * s') with s' its outputs per thread; threads:
  bx * by.
* 2-D VALU family (Fig. 4's kernel with outputs per work-item along M too):
  program parameters bx, by, s (outputs per work-item along N), sy (along
  M), bk (the LDS tiles' K extent, free of by); programs {} and {gran} (one
  output per work-item, s = sy = 1).  LDS bytes: 4 * (by * sy' * (bk + 4) +
  bk * bx * s') (A rows padded to bk + 4 elements, a 16-byte multiple);
  threads: bx * by.
* MFMA family: program parameters bm, bn, bk, wm, wn; programs {} (two LDS
  stages) and {single} (one).  One stage holds, in float32, an A tile bm x
  (bk + 4) and a B tile bk x (bn + 4); in bfloat16 an A tile bm x (bk + 8) and
  a B tile bk x (bn + 32); in int32 (four one-byte digit planes per operand,
  rows of bk + 16 bytes) 4 * (bm + bn) * (bk + 16) bytes; threads:
  64 * wm * wn.
* Transposition family (Section 5.2, Fig. 7): program parameters bx (the
  paper's B1), by (B0), s; programs as in the VALU family; the cached program
  holds one (by * s') x bx tile padded by one element per row: 4 * (by * s')
  * (bx + 1) bytes; threads bx * by.  One compiled program serves every
  4-byte element type.
* Matrix-addition family (Section 1, Fig. 1 and Fig. 2): program parameters
  bx (the paper's B1), by (B0), s; programs {} (s elements per thread) and
  {gran} (one); no LDS, so the counters are registers per workgroup and
  threads per workgroup (bx * by) only, the two machine parameters of Fig. 2.
* 1D Jacobi family (Section 5, Fig. 6): program parameters B (work-items
  per workgroup) and s (points per work-item); programs as in the VALU
  family; the cached program holds the tile's s' * B inputs and one halo
  point on each side: 4 * (s' * B + 2) bytes; threads B.
* Polynomial-division family (Section 5, Fig. 8): program parameters B and s
  as the 1D Jacobi family; the cached program holds the tile's s' * B values
  of a and of b and the leading coefficient: 4 * (2 * s' * B + 1) bytes;
  threads B; 32-bit residues only (stored under the int32 dtype).
* An MFMA program also exists as an element-load twin (rows not aligned for
  16-byte loads) and, up to 512 work-items, as a split form running a share
  of K; the program's registers are the largest of its kernels' (any of them
  may run it).
* Registers of a workgroup: each lane of a wavefront allocates its VGPRs
  rounded up to 4 plus its AGPRs, rounded up to 8 (gfx950's unified register
  file); a workgroup occupies ceil(threads / 64) wavefronts of 64 lanes.  The
  VGPR/AGPR counts per compiled instance are input data (the compiler's
  report), not derived here.

Properties checked (Definition 3 and Section 3.7): completeness (coverage),
soundness of the selected program, no dead leaves, optimality of each
counter at some leaf, preference for the unmodified program where it fits,
and the tree-height bound.
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Tuple

import numpy as np

from . import comprehensive as co

F32, I32, BF16 = 0, 1, 2
VALU, MFMA, TRANSPOSE, MADD, JACOBI, POLYDIV, VALU2 = 0, 1, 2, 3, 4, 5, 6
GRAN, NOLDS = 1, 2          # VALU strategy bits
SINGLE = 1                  # MFMA strategy bit
ELEMENT = 4                 # MFMA: the twin instance reading rows element by element
SPLIT = 16                  # MFMA: the form running a share of K (products split along K)

VALU_VARIANTS = (0, GRAN, GRAN | NOLDS, NOLDS)
MFMA_VARIANTS = (0, SINGLE)
MADD_VARIANTS = (0, GRAN)
VALU2_VARIANTS = (0, GRAN)

# machine grid: LDS bytes per workgroup, registers per workgroup, threads per workgroup
LDS_GRID = (4 * 1024, 16 * 1024, 48 * 1024, 64 * 1024, 160 * 1024)
REG_GRID = (16384, 32768, 65536, 131072)
THREAD_GRID = (256, 512, 1024)


def regs_per_block(vgpr: int, agpr: int, threads: int) -> int:
    per_lane = -(-(-(-vgpr // 4) * 4 + agpr) // 8) * 8
    waves = -(-threads // 64)
    return per_lane * 64 * waves


def valu_lds(variant: int, bx: int, by: int, s: int) -> int:
    if variant & NOLDS:
        return 0
    outs = 1 if variant & GRAN else s
    bk = by
    return 4 * (by * (bk + 1) + bk * bx * outs)


def valu2_lds(variant: int, bx: int, by: int, s: int, sy: int, bk: int) -> int:
    outs, rows = (1, 1) if variant & GRAN else (s, sy)
    return 4 * (by * rows * (bk + 4) + bk * bx * outs)


def transpose_lds(variant: int, bx: int, by: int, s: int) -> int:
    if variant & NOLDS:
        return 0
    outs = 1 if variant & GRAN else s
    return 4 * by * outs * (bx + 1)


def jacobi_lds(variant: int, b: int, s: int) -> int:
    if variant & 4:             # several steps per launch: two windows with a 16-point halo each side
        return 8 * (s * b + 32)
    if variant & NOLDS:
        return 0
    outs = 1 if variant & GRAN else s
    return 4 * (outs * b + 2)


FUSED = 4                   # polynomial division: the one-launch program


def polydiv_lds(variant: int, b: int, s: int) -> int:
    if variant & FUSED:         # quotient, top of b, b window of a tile
        return 4 * (3 * 1024 + s * b)
    if variant & NOLDS:
        return 0
    outs = 1 if variant & GRAN else s
    return 4 * (2 * outs * b + 1)


def mfma_lds(dtype: int, variant: int, bm: int, bn: int, bk: int) -> int:
    stages = 1 if variant & SINGLE else 2
    if dtype == F32:
        one = 4 * (bm * (bk + 4) + bk * (bn + 4))
    elif dtype == I32:
        one = 4 * (bm + bn) * (bk + 16)
    else:
        one = 2 * (bm * (bk + 8) + bk * (bn + 32))
    return stages * one


class InstanceData:
    """Per-instance register counts taken from the library's description."""

    def __init__(self, instances: List[dict]):
        self.by_key = {}
        for e in instances:
            if e["family"] == VALU2:
                key = (VALU2, e["dtype"], e["variant"], e["bx"], e["by"], e["s"], e["sy"], e["bk"])
            elif e["family"] in (VALU, TRANSPOSE, MADD, JACOBI, POLYDIV):
                key = (e["family"], e["dtype"], e["variant"], e["bx"], e["by"], e["s"])
            else:
                key = (MFMA, e["dtype"], e["variant"], e["bm"], e["bn"], e["bk"], e["wm"], e["wn"])
            self.by_key[key] = e

    def regs(self, family: int, dtype: int, variant: int, point: Tuple[int, ...]):
        if family == VALU2:
            bx, by, s, sy, bk = point
            outs, rows = (1, 1) if variant & GRAN else (s, sy)
            e = self.by_key.get((VALU2, dtype, 0, bx, by, outs, rows, bk))
        elif family in (JACOBI, POLYDIV):
            b, s = point
            outs = 1 if variant & GRAN else s
            e = self.by_key.get((family, dtype, variant & NOLDS, b, 1, outs))
        elif family in (VALU, TRANSPOSE, MADD):
            bx, by, s = point
            kernel = variant & NOLDS
            outs = 1 if variant & GRAN else s
            dt = F32 if family == TRANSPOSE else dtype
            e = self.by_key.get((family, dt, kernel, bx, by, outs))
        else:
            e = self.by_key.get((MFMA, dtype, variant & SINGLE) + tuple(point))
            forms = [self.by_key.get((MFMA, dtype, (variant & SINGLE) | f) + tuple(point)) for f in (ELEMENT, SPLIT)]
            if e is not None and "vgpr" in e:
                return max(regs_per_block(k["vgpr"], k["agpr"], k["threads"]) for k in [e] + forms if k is not None)
        if e is None or "vgpr" not in e:
            return None
        return regs_per_block(e["vgpr"], e["agpr"], e["threads"])


def threads(family: int, point) -> int:
    if family in (JACOBI, POLYDIV):
        return point[0]
    if family in (VALU, TRANSPOSE, MADD, VALU2):
        return point[0] * point[1]
    return 64 * point[3] * point[4]


def lds(family: int, dtype: int, variant: int, point) -> int:
    if family == VALU:
        return valu_lds(variant, *point)
    if family == VALU2:
        return valu2_lds(variant, *point)
    if family == TRANSPOSE:
        return transpose_lds(variant, *point)
    if family == MADD:
        return 0
    if family == JACOBI:
        return jacobi_lds(variant, *point)
    if family == POLYDIV:
        return polydiv_lds(variant, *point)
    return mfma_lds(dtype, variant, point[0], point[1], point[2])


def fits(inst: InstanceData, family, dtype, variant, point, Z, V, T) -> bool:
    r = inst.regs(family, dtype, variant, point)
    if r is None:
        return False
    return lds(family, dtype, variant, point) <= Z and r <= V and threads(family, point) <= T


def variants(family: int):
    if family == MADD:
        return MADD_VARIANTS
    if family == VALU2:
        return VALU2_VARIANTS
    return MFMA_VARIANTS if family == MFMA else VALU_VARIANTS


def machine_grid():
    return list(itertools.product(LDS_GRID, REG_GRID, THREAD_GRID))


# ---------------------------------------------------------------------------
# the same families as code fragments for Algorithms 1 and 2 (oracle side)


def oracle_family(family: int, dtype: int, points: List[Tuple[int, ...]], inst: InstanceData) -> co.Family:
    """The family as a code fragment: counters r_Z (LDS bytes, limit Z), r_V
    (registers per workgroup, limit V, a table symbol per program), r_T
    (threads, limit T), in that gamma order; strategies in omega order.
    Machine-symbol domains hold every threshold value a counter takes (and
    its predecessor), 0, and one value above all of them, so the finite
    enumeration decides the same as integers without bound."""
    pts = [tuple(p) for p in points]
    if family == MADD:
        return _madd_family(dtype, pts, inst)
    if family in (JACOBI, POLYDIV):
        program = ["B", "s"]
        strategies = [co.Strategy("gran", False, frozenset({"r_Z", "r_V"})),
                      co.Strategy("nolds", False, frozenset({"r_Z", "r_V"}))]
        names = {0: "rho_tiled", GRAN: "rho_tiled_s1", NOLDS: "rho_direct", GRAN | NOLDS: "rho_direct_s1"}

        def lds_poly(applied):
            a = set(applied)
            if "nolds" in a:
                return co.Poly.const(0)
            if family == POLYDIV:
                return co.parse_poly("8*B + 4") if "gran" in a else co.parse_poly("8*s*B + 4")
            if "gran" in a:
                return co.parse_poly("4*B + 8")
            return co.parse_poly("4*s*B + 8")

        def bits(applied):
            a = set(applied)
            return (GRAN if "gran" in a else 0) | (NOLDS if "nolds" in a else 0)

        thr = co.parse_poly("B")
    elif family == TRANSPOSE:
        program = ["bx", "by", "s"]
        strategies = [co.Strategy("gran", False, frozenset({"r_Z", "r_V"})),
                      co.Strategy("nolds", False, frozenset({"r_Z", "r_V"}))]
        names = {0: "rho_tiled", GRAN: "rho_tiled_s1", NOLDS: "rho_direct", GRAN | NOLDS: "rho_direct_s1"}

        def lds_poly(applied):
            a = set(applied)
            if "nolds" in a:
                return co.Poly.const(0)
            if "gran" in a:
                return co.parse_poly("4*by*(bx+1)")
            return co.parse_poly("4*by*s*(bx+1)")

        def bits(applied):
            a = set(applied)
            return (GRAN if "gran" in a else 0) | (NOLDS if "nolds" in a else 0)

        thr = co.parse_poly("bx*by")
    elif family == VALU2:
        program = ["bx", "by", "s", "sy", "bk"]
        strategies = [co.Strategy("gran", False, frozenset({"r_Z", "r_V"}))]
        names = {0: "rho_tiled", GRAN: "rho_tiled_s1"}

        def lds_poly(applied):
            if "gran" in applied:
                return co.parse_poly("4*(by*(bk+4) + bk*bx)")
            return co.parse_poly("4*(by*sy*(bk+4) + bk*bx*s)")

        def bits(applied):
            return GRAN if "gran" in applied else 0

        thr = co.parse_poly("bx*by")
    elif family == VALU:
        program = ["bx", "by", "s"]
        strategies = [co.Strategy("gran", False, frozenset({"r_Z", "r_V"})),
                      co.Strategy("nolds", False, frozenset({"r_Z", "r_V"}))]
        names = {0: "rho_tiled", GRAN: "rho_tiled_s1", NOLDS: "rho_direct", GRAN | NOLDS: "rho_direct_s1"}

        def lds_poly(applied):
            a = set(applied)
            if "nolds" in a:
                return co.Poly.const(0)
            if "gran" in a:
                return co.parse_poly("4*(by*(by+1) + by*bx)")
            return co.parse_poly("4*(by*(by+1) + by*bx*s)")

        def bits(applied):
            a = set(applied)
            return (GRAN if "gran" in a else 0) | (NOLDS if "nolds" in a else 0)

        thr = co.parse_poly("bx*by")
    else:
        program = ["bm", "bn", "bk", "wm", "wn"]
        strategies = [co.Strategy("single", False, frozenset({"r_Z", "r_V"}))]
        names = {0: "rho_two_stage", SINGLE: "rho_one_stage"}
        one = co.parse_poly({F32: "4*(bm*(bk+4) + bk*(bn+4))", I32: "4*(bm+bn)*(bk+16)"}.get(
            dtype, "2*(bm*(bk+8) + bk*(bn+32))"))

        def lds_poly(applied):
            return one if "single" in applied else co.Poly.const(2) * one

        def bits(applied):
            return SINGLE if "single" in applied else 0

        thr = co.parse_poly("64*wm*wn")

    counters = [co.Counter("r_Z", "resource", "Z", lds_poly),
                co.Counter("r_V", "resource", "V", lambda applied: co.Poly.sym(names[bits(applied)])),
                co.Counter("r_T", "resource", "T", lambda applied: thr)]

    def table_fn(var):
        def f(env):
            cols = [env[s] for s in program]
            out = []
            for p in zip(*cols):
                r = inst.regs(family, dtype, var, tuple(int(x) for x in p))
                out.append(r if r is not None else 1 << 40)
            return np.array(out, dtype=np.int64)
        return f

    tables = {names[v]: table_fn(v) for v in names}
    thresholds_z, thresholds_v, thresholds_t = {0}, {0}, {0}
    for p in pts:
        for v in variants(family):
            z = lds(family, dtype, v, p)
            thresholds_z |= {z, max(z - 1, 0)}
            r = inst.regs(family, dtype, v, p)
            if r is not None:
                thresholds_v |= {r, max(r - 1, 0)}
        t = threads(family, p)
        thresholds_t |= {t, t - 1}
    doms: Dict[str, list] = {
        "Z": sorted(thresholds_z | {max(thresholds_z) + 1}),
        "V": sorted(thresholds_v | {max(thresholds_v) + 1}),
        "T": sorted(thresholds_t | {max(thresholds_t) + 1}),
    }
    for k, name in enumerate(program):
        doms[name] = sorted({p[k] for p in pts})
    return co.Family(machine=["Z", "V", "T"], program=program, data=[], counters=counters,
                     strategies=strategies, domains=doms, tables=tables, points=pts)


def _madd_family(dtype: int, pts, inst: InstanceData) -> co.Family:
    """Fig. 2's system as a code fragment: counters r_V (registers per
    workgroup, a table symbol per program) and r_T (bx * by), in that order;
    one strategy, granularity reduction, which lowers r_V."""
    program = ["bx", "by", "s"]
    names = {0: "rho", GRAN: "rho_s1"}
    counters = [co.Counter("r_V", "resource", "V",
                           lambda applied: co.Poly.sym(names[GRAN if "gran" in applied else 0])),
                co.Counter("r_T", "resource", "T", lambda applied: co.parse_poly("bx*by"))]
    strategies = [co.Strategy("gran", False, frozenset({"r_V"}))]

    def table_fn(var):
        def f(env):
            out = []
            for p in zip(*[env[s] for s in program]):
                r = inst.regs(MADD, dtype, var, tuple(int(x) for x in p))
                out.append(r if r is not None else 1 << 40)
            return np.array(out, dtype=np.int64)
        return f

    thresholds_v, thresholds_t = {0}, {0}
    for p in pts:
        for v in MADD_VARIANTS:
            r = inst.regs(MADD, dtype, v, p)
            if r is not None:
                thresholds_v |= {r, max(r - 1, 0)}
        t = threads(MADD, p)
        thresholds_t |= {t, t - 1}
    doms: Dict[str, list] = {"V": sorted(thresholds_v | {max(thresholds_v) + 1}),
                             "T": sorted(thresholds_t | {max(thresholds_t) + 1})}
    for k, name in enumerate(program):
        doms[name] = sorted({p[k] for p in pts})
    return co.Family(machine=["V", "T"], program=program, data=[], counters=counters,
                     strategies=strategies, domains=doms, tables={names[v]: table_fn(v) for v in names},
                     points=pts)
