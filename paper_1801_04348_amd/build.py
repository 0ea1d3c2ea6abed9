"""Builds libpk.so for gfx950.

Steps:
  1. generate the kernel-instance translation units (one extern "C" kernel per
     program-parameter point and variant of each family) and their registry;
  2. compile them with hipcc in parallel, with the compiler's
     kernel-resource-usage report switched on;
  3. parse that report (VGPRs, AGPRs, SGPRs, scratch, LDS per kernel) into a
     generated resource table -- the register counts the case table's
     register counter reads;
  4. compile the host sources and link everything into
     paper_1801_04348_amd/libpk.so.

Every HIP translation unit is built with packed FP32 instructions disabled
(-target-feature -packed-fp32-ops).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
GEN = os.path.join(BUILD, "gen")
LIB = os.path.join(PKG, "libpk.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-I", INCLUDE, "-I", CSRC,
          "-Wno-unused-command-line-argument"]
DEVICE = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Rpass-analysis=kernel-resource-usage"]
HOST_SOURCES = ["engine.cpp", "families.cpp", "capi.cpp", "select.cpp", "registry.cpp", "grouped.cpp", "transpose.cpp",
                "madd.cpp", "jacobi.cpp"]
DEVICE_SOURCES = ["costmodel.hip", "polydiv.hip", "probes.hip", "fill.hip", "noalloc.hip"]

F32, I32, BF16 = 0, 1, 2
DT_NAME = {F32: "f32", I32: "i32", BF16: "bf16"}
DT_CTYPE = {F32: "float", I32: "int32_t"}
FAM_VALU, FAM_MFMA, FAM_TR, FAM_MA, FAM_JA, FAM_PD, FAM_VALU2 = 0, 1, 2, 3, 4, 5, 6
VALU_GRAN, VALU_NOLDS = 1, 2
MFMA_SINGLE = 1
MFMA_GROUPED = 2
MFMA_ELEMENT = 4
MFMA_MIXED = 8
MFMA_SPLIT = 16
# the mixed grouped kernels' tile programs (csrc/kernels/kargs.hpp kMixedTile,
# in the same order) and K tiles
MIXED_TILES = [(64, 64), (128, 64), (64, 128), (128, 128)]
MIXED_BK = {0: 32, 2: 64}

# program-parameter domains (the families' point sets)
VALU_B = (4, 8, 16, 32)
VALU_S = (1, 2, 4, 8)
VALU2_S = (2, 4)      # outputs per work-item along N and along M
VALU2_BK = (16, 32)   # K extent of the LDS tiles
JA_B = (16, 32, 64, 128, 256, 512, 1024)
JA_S = (1, 2, 4, 8)
MA_BX = (64, 128, 256)
MA_BY = (1, 2, 4)
MA_S = (1, 2, 4, 8)
TR_BX = (16, 32, 64)
TR_BY = (4, 8, 16, 32)
TR_S = (1, 2, 4, 8)
MFMA_F32 = [(64, 64, 32, 2, 2), (128, 64, 32, 2, 2), (64, 128, 32, 2, 2), (128, 128, 32, 2, 2),
            (256, 128, 32, 4, 2), (128, 256, 32, 2, 4), (256, 256, 32, 4, 4), (256, 128, 32, 2, 2),
            (128, 256, 32, 2, 2), (256, 128, 16, 4, 2), (128, 256, 16, 2, 4)]
MFMA_BF16 = [(64, 64, 64, 2, 2), (128, 64, 64, 2, 2), (64, 128, 64, 2, 2), (128, 128, 64, 2, 2),
             (256, 128, 64, 4, 2), (128, 256, 64, 2, 4), (256, 256, 64, 4, 4),
             (256, 128, 32, 2, 2), (128, 256, 32, 2, 2), (256, 128, 64, 2, 2), (128, 256, 64, 2, 2)]

# int32 on the int8 matrix cores (four signed digit planes per operand)
MFMA_I32 = [(64, 64, 32, 2, 2), (128, 64, 32, 2, 2), (64, 128, 32, 2, 2), (64, 64, 64, 2, 2)]


def valu_lds(bx, by, s, nolds):
    return 0 if nolds else 4 * (by * (by + 1) + by * bx * s)


def valu2_lds(bx, by, sx, sy, bk):
    return 4 * (by * sy * (bk + 4) + bk * bx * sx)


def mfma_reg_cap(dt, threads, stages, kind, bm=0, bn=0):
    """At most 65536 / threads registers a lane, so that the workgroup fits a
    block register budget of 65536 (the smaller figure HIP runtimes report for
    gfx950), where the compiler's own choice would exceed it and the capped
    program compiles without spilling: element-load twins and grouped programs
    of 256 work-items (256 registers; their loads at chosen addresses hold
    more), programs of 256 work-items with tiles larger than 128 x 128 (256),
    and single-stage float32 programs of 512 (128)."""
    if (dt == F32 and threads == 512 and stages == 1) or (kind != "wide" and threads == 256) or \
            (threads == 256 and bm * bn > 128 * 128):
        return "__attribute__((amdgpu_waves_per_eu(%d)))" % (threads // 128)
    return ""


def twinless_bf16(bm, bn, bk, wm, wn):
    """bfloat16 programs built without an element-load twin (it would spill)."""
    return bm * bn >= 256 * 256 or (bk == 64 and wm * wn == 4 and bm * bn >= 128 * 256)


def mfma_lds(dtype, bm, bn, bk, stages):
    if dtype == F32:
        return stages * 4 * (bm * (bk + 4) + bk * (bn + 4))
    if dtype == I32:
        return stages * 4 * (bm + bn) * (bk + 16)
    return stages * 2 * (bm * (bk + 8) + bk * (bn + 32))


def instances():
    """(tu_group, name, macro_call, entry_fields) for every kernel instance."""
    out = []
    for dt in (F32, I32):
        for bx in VALU_B:
            for by in VALU_B:
                for s in VALU_S:
                    for nolds in (0, 1):
                        kind = "direct" if nolds else "tiled"
                        name = "pk_valu_%s_%s_bx%d_by%d_s%d" % (kind, DT_NAME[dt], bx, by, s)
                        if nolds:
                            body = "pkk::valu_direct<%s, %d, %d, %d>(a);" % (DT_CTYPE[dt], bx, by, s)
                        else:
                            body = "pkk::valu_tiled<%s, %d, %d, %d, %d>(a);" % (DT_CTYPE[dt], bx, by, s, by)
                        entry = dict(family=FAM_VALU, variant=VALU_NOLDS if nolds else 0, dtype=dt,
                                     bx=bx, by=by, s=s, bk=by, bm=0, bn=0, wm=0, wn=0, threads=bx * by,
                                     lds=valu_lds(bx, by, s, nolds), tile_m=by, tile_n=bx * s)
                        out.append(("valu_%s_by%d" % (DT_NAME[dt], by), name, body, entry))
    # 2-D micro-tile VALU programs: workgroups of one to four wavefronts; the
    # one-output program of each workgroup and K extent (granularity reduction)
    for dt in (F32, I32):
        for bx in VALU_B:
            for by in VALU_B:
                if not 64 <= bx * by <= 256:
                    continue
                for bk in VALU2_BK:
                    for sx, sy in [(1, 1)] + [(a, b) for a in VALU2_S for b in VALU2_S]:
                        name = "pk_valu2_%s_bx%d_by%d_s%dx%d_bk%d" % (DT_NAME[dt], bx, by, sy, sx, bk)
                        body = "pkk::valu_tiled2<%s, %d, %d, %d, %d, %d>(a);" % (DT_CTYPE[dt], bx, by, sx, sy, bk)
                        entry = dict(family=FAM_VALU2, variant=0, dtype=dt, bx=bx, by=by, s=sx, sy=sy, bk=bk, bm=0,
                                     bn=0, wm=0, wn=0, threads=bx * by, lds=valu2_lds(bx, by, sx, sy, bk),
                                     tile_m=by * sy, tile_n=bx * sx)
                        out.append(("valu2_%s_bx%d" % (DT_NAME[dt], bx), name, body, entry))
    for dt, cfgs, fn in ((F32, MFMA_F32, "mfma_f32"), (BF16, MFMA_BF16, "mfma_bf16")):
        for (bm, bn, bk, wm, wn) in cfgs:
            for stages in (2, 1):
                name = "pk_mfma_%s_%dx%dx%d_w%dx%d_st%d" % (DT_NAME[dt], bm, bn, bk, wm, wn, stages)
                body = "pkk::%s<%d, %d, %d, %d, %d, %d>(a);" % (fn, bm, bn, bk, wm, wn, stages)
                entry = dict(family=FAM_MFMA, variant=0 if stages == 2 else MFMA_SINGLE, dtype=dt,
                             bx=0, by=0, s=0, bk=bk, bm=bm, bn=bn, wm=wm, wn=wn, threads=64 * wm * wn,
                             lds=mfma_lds(dt, bm, bn, bk, stages), tile_m=bm, tile_n=bn)
                entry["attrs"] = mfma_reg_cap(dt, 64 * wm * wn, stages, "wide", bm, bn)
                out.append(("mfma_%s_%d" % (DT_NAME[dt], bm * 1000 + bn), name, body, entry))
                # the split-along-K form of the wide program (workgroups of up
                # to 512 work-items; not the single-stage float32 programs of
                # 512, whose 128-register cap it would exceed, nor those of
                # 128 x 256 outputs or more, whose split form would spill)
                if 64 * wm * wn <= 512 and not (dt == F32 and stages == 1 and
                                                (64 * wm * wn == 512 or bm * bn >= 128 * 256)):
                    body_sk = "pkk::%s<%d, %d, %d, %d, %d, %d, true, true>(a);" % (fn, bm, bn, bk, wm, wn, stages)
                    entry_sk = dict(entry, variant=entry["variant"] | MFMA_SPLIT)
                    out.append(("mfma_%s_%d_sk" % (DT_NAME[dt], bm * 1000 + bn), name + "_sk", body_sk, entry_sk))
                # the element-load twin, launched for rows not aligned for 16-byte
                # loads (none for the bf16 tiles whose twin would spill: the
                # largest, and those of K tile 64 on four wavefronts with 128 x
                # 256 outputs)
                if dt == BF16 and twinless_bf16(bm, bn, bk, wm, wn):
                    continue
                body_el = "pkk::%s<%d, %d, %d, %d, %d, %d, false>(a);" % (fn, bm, bn, bk, wm, wn, stages)
                entry_el = dict(entry, variant=entry["variant"] | MFMA_ELEMENT,
                                attrs=mfma_reg_cap(dt, 64 * wm * wn, stages, "twin", bm, bn))
                # (a translation unit of its own: compiled beside the wide kernel
                # it changes the wide kernel's instruction schedule, measurably)
                out.append(("mfma_%s_%d_el" % (DT_NAME[dt], bm * 1000 + bn), name + "_el", body_el, entry_el))
    # int32 on the int8 matrix cores: a wide form (16-byte loads of A where its
    # rows are aligned) and its element-load twin; no split form.  Wave tiles
    # of two 32 x 32 blocks hold 128 accumulator registers (four sums per
    # block): those programs are capped at 256 registers a lane, the block
    # budget of 65536 over 256 work-items.
    for (bm, bn, bk, wm, wn) in MFMA_I32:
        cap = "__attribute__((amdgpu_waves_per_eu(2)))" if bm * bn > 64 * 64 else ""
        for stages in (2, 1):
            name = "pk_mfma_i32_%dx%dx%d_w%dx%d_st%d" % (bm, bn, bk, wm, wn, stages)
            entry = dict(family=FAM_MFMA, variant=0 if stages == 2 else MFMA_SINGLE, dtype=I32,
                         bx=0, by=0, s=0, bk=bk, bm=bm, bn=bn, wm=wm, wn=wn, threads=64 * wm * wn,
                         lds=mfma_lds(I32, bm, bn, bk, stages), tile_m=bm, tile_n=bn, attrs=cap)
            body = "pkk::mfma_i32<%d, %d, %d, %d, %d, %d>(a);" % (bm, bn, bk, wm, wn, stages)
            out.append(("mfma_i32", name, body, entry))
            body_el = "pkk::mfma_i32<%d, %d, %d, %d, %d, %d, false>(a);" % (bm, bn, bk, wm, wn, stages)
            entry_el = dict(entry, variant=entry["variant"] | MFMA_ELEMENT)
            out.append(("mfma_i32_el", name + "_el", body_el, entry_el))
    # transposition: tiled and direct programs (bit copies of 4-byte elements)
    for bx in TR_BX:
        for by in TR_BY:
            if bx * by > 1024:
                continue
            for s in TR_S:
                for nolds in (0, 1):
                    kind = "direct" if nolds else "tiled"
                    name = "pk_transpose_%s_bx%d_by%d_s%d" % (kind, bx, by, s)
                    body = "pkk::transpose_%s<%d, %d, %d>(a);" % (kind, by, bx, s)
                    entry = dict(family=FAM_TR, variant=VALU_NOLDS if nolds else 0, dtype=F32, bx=bx, by=by, s=s,
                                 bk=0, bm=0, bn=0, wm=0, wn=0, threads=bx * by,
                                 lds=0 if nolds else 4 * by * s * (bx + 1), tile_m=by * s, tile_n=bx,
                                 args="pkk::TrArgs a")
                    out.append(("transpose_bx%d" % bx, name, body, entry))
    # matrix addition
    for dt in (F32, I32):
        for bx in MA_BX:
            for by in MA_BY:
                for s in MA_S:
                    name = "pk_madd_%s_bx%d_by%d_s%d" % (DT_NAME[dt], bx, by, s)
                    body = "pkk::madd<%s, %d, %d, %d>(a);" % (DT_CTYPE[dt], bx, by, s)
                    entry = dict(family=FAM_MA, variant=0, dtype=dt, bx=bx, by=by, s=s, bk=0, bm=0, bn=0, wm=0,
                                 wn=0, threads=bx * by, lds=0, tile_m=by, tile_n=bx * s, args="pkk::MaArgs a")
                    out.append(("madd_%s" % DT_NAME[dt], name, body, entry))
    # 1D Jacobi: cached (LDS) and direct programs
    for dt in (F32, I32):
        for nolds in (False, True):
            for b in JA_B:
                for s in JA_S:
                    kind = "direct" if nolds else "tiled"
                    name = "pk_jacobi_%s_%s_b%d_s%d" % (kind, DT_NAME[dt], b, s)
                    body = "pkk::jacobi_%s<%s, %d, %d>(a);" % (kind, DT_CTYPE[dt], b, s)
                    lds = 0 if nolds else 4 * (s * b + 2)
                    entry = dict(family=FAM_JA, variant=VALU_NOLDS if nolds else 0, dtype=dt, bx=b, by=1, s=s, bk=0,
                                 bm=0, bn=0, wm=0, wn=0, threads=b, lds=lds, tile_m=1, tile_n=s * b,
                                 args="pkk::JaArgs a")
                    out.append(("jacobi_%s" % DT_NAME[dt], name, body, entry))
    # 1D Jacobi: several steps per launch (odd step counts, up to 15)
    for dt in (F32, I32):
        for b in (256, 512, 1024):
            for s in (1, 2, 4):
                name = "pk_jacobi_fused_%s_b%d_s%d" % (DT_NAME[dt], b, s)
                body = "pkk::jacobi_fused<%s, %d, %d>(a);" % (DT_CTYPE[dt], b, s)
                entry = dict(family=FAM_JA, variant=4, dtype=dt, bx=b, by=1, s=s, bk=0, bm=0, bn=0, wm=0, wn=0,
                             threads=b, lds=2 * 4 * (s * b + 2 * 16), tile_m=1, tile_n=s * b, args="pkk::JfArgs a")
                out.append(("jacobi_fused", name, body, entry))
    # polynomial division steps: cached (LDS) and direct programs, 32-bit residues
    for nolds in (False, True):
        for b in JA_B:
            for s in JA_S:
                kind = "direct" if nolds else "tiled"
                name = "pk_polydiv_%s_b%d_s%d" % (kind, b, s)
                body = "pkk::polydiv_step_%s<%d, %d>(a);" % (kind, b, s)
                entry = dict(family=FAM_PD, variant=VALU_NOLDS if nolds else 0, dtype=I32, bx=b, by=1, s=s, bk=0,
                             bm=0, bn=0, wm=0, wn=0, threads=b, lds=0 if nolds else 4 * (2 * s * b + 1),
                             tile_m=1, tile_n=s * b, args="pkk::PdArgs a")
                out.append(("polydiv_steps", name, body, entry))
    # one-launch polynomial division (quotient recurrence, then the remainder)
    for b in (64, 128, 256, 512, 1024):
        for s in JA_S:
            for r in (2, 16):
                name = "pk_polydiv_fused_b%d_s%d_k%d" % (b, s, 64 * r)
                body = "pkk::polydiv_fused<%d, %d, %d>(a);" % (b, s, r)
                entry = dict(family=FAM_PD, variant=4 | (8 if r == 16 else 0), dtype=I32, bx=b, by=1, s=s, bk=0,
                             bm=0, bn=0, wm=0, wn=0, threads=b, lds=4 * (3 * 1024 + s * b), tile_m=1, tile_n=s * b,
                             args="pkk::PdArgs a")
                out.append(("polydiv_fused", name, body, entry))
    # persistent grouped instances of the MFMA programs up to 128 x 128
    gfn = {F32: "grouped_f32", BF16: "grouped_bf16"}
    for dt, cfgs in ((F32, MFMA_F32), (BF16, MFMA_BF16)):
        for (bm, bn, bk, wm, wn) in cfgs:
            if bm > 128 or bn > 128:
                continue
            for stages in (2, 1):
                if dt == BF16 and bm * bn >= 128 * 128 and stages == 2:
                    continue  # would spill at 256 registers a lane (its loads at chosen addresses hold more)
                # the wide kernel (rows aligned for 16-byte loads) and its
                # element-load twin, for the products whose rows are not
                for wide in (True, False):
                    name = "pk_grouped_%s_%dx%dx%d_w%dx%d_st%d%s" % (DT_NAME[dt], bm, bn, bk, wm, wn, stages,
                                                                   "" if wide else "_el")
                    body = "pkk::%s<%d, %d, %d, %d, %d, %d, %s>(g);" % (gfn[dt], bm, bn, bk, wm, wn, stages,
                                                                       "true" if wide else "false")
                    entry = dict(family=FAM_MFMA, variant=MFMA_GROUPED | (0 if stages == 2 else MFMA_SINGLE) |
                                 (0 if wide else MFMA_ELEMENT), dtype=dt, bx=0, by=0, s=0, bk=bk, bm=bm, bn=bn,
                                 wm=wm, wn=wn, threads=64 * wm * wn, lds=mfma_lds(dt, bm, bn, bk, stages), tile_m=bm,
                                 tile_n=bn, args="pkk::GroupArgs g",
                                 attrs=mfma_reg_cap(dt, 64 * wm * wn, stages, "grouped"))
                    out.append(("grouped_%s%s" % (DT_NAME[dt], "" if wide else "_el"), name, body, entry))
    # mixed grouped kernels: a tile program per product (kMixedTile), 2 x 2
    # wavefronts, LDS sized for the largest program
    for dt, fn in ((F32, "grouped_mixed_f32"), (BF16, "grouped_mixed_bf16")):
        bk = MIXED_BK[dt]
        bm, bn = max(MIXED_TILES, key=lambda t: t[0] * t[1])
        for stages in ((2, 1) if dt == F32 else (1,)):  # bf16: its 128 x 128 program spills with two stages
            for wide in (True, False):
                name = "pk_grouped_mixed_%s_w2x2_st%d%s" % (DT_NAME[dt], stages, "" if wide else "_el")
                body = "pkk::%s<%d, %s>(g);" % (fn, stages, "true" if wide else "false")
                lds = max(mfma_lds(dt, m, n, bk, stages) for m, n in MIXED_TILES)
                entry = dict(family=FAM_MFMA, variant=MFMA_GROUPED | MFMA_MIXED | (0 if stages == 2 else MFMA_SINGLE) |
                             (0 if wide else MFMA_ELEMENT), dtype=dt, bx=0, by=0, s=0, bk=bk, bm=bm, bn=bn, wm=2,
                             wn=2, threads=256, lds=lds, tile_m=bm, tile_n=bn, args="pkk::GroupArgs g",
                             attrs=mfma_reg_cap(dt, 256, stages, "grouped"))
                out.append(("grouped_mixed_%s%s" % (DT_NAME[dt], "" if wide else "_el"), name, body, entry))
    return out


def _entry_c(name, e):
    return ('    {"%s", (const void *)&%s, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d},'
            % (name, name, e["family"], e["variant"], e["dtype"], e["bx"], e["by"], e["s"], e["bk"],
               e["bm"], e["bn"], e["wm"], e["wn"], e["threads"], e["lds"], e["tile_m"], e["tile_n"],
               e.get("sy", 0)))


def generate():
    os.makedirs(GEN, exist_ok=True)
    groups = {}
    for grp, name, body, entry in instances():
        groups.setdefault(grp, []).append((name, body, entry))
    tus = []
    for grp, items in sorted(groups.items()):
        lines = ["// generated by build.py -- kernel instances of group %s" % grp,
                 "#include <hip/hip_runtime.h>", '#include "kernels/valu.hpp"', '#include "kernels/mfma.hpp"', '#include "kernels/mfma_i32.hpp"',
                 '#include "kernels/transpose.hpp"', '#include "kernels/madd.hpp"',
                 '#include "kernels/jacobi.hpp"', '#include "kernels/polydiv.hpp"', ""]
        for name, body, entry in items:
            arg = entry.get("args", "pkk::MmArgs a")
            attrs = entry.get("attrs", "")
            lines.append('extern "C" __global__ void __launch_bounds__(%d) %s%s(%s) { %s }'
                         % (entry["threads"], attrs + " " if attrs else "", name, arg, body))
        lines.append("")
        lines.append("static const pkk::KernelEntry entries[] = {")
        for name, body, entry in items:
            lines.append(_entry_c(name, entry))
        lines.append("};")
        lines.append('extern "C" const pkk::KernelEntry *pk_gen_%s(int *n) {' % grp)
        lines.append("    *n = (int)(sizeof entries / sizeof entries[0]);")
        lines.append("    return entries;")
        lines.append("}")
        path = os.path.join(GEN, grp + ".hip")
        _write_if_changed(path, "\n".join(lines) + "\n")
        tus.append((grp, path))
    reg = ["// generated by build.py -- concatenation of the instance groups",
           "#include <vector>", '#include "kernels/kargs.hpp"', ""]
    for grp, _ in tus:
        reg.append('extern "C" const pkk::KernelEntry *pk_gen_%s(int *n);' % grp)
    reg.append('extern "C" const pkk::KernelEntry *pk_gen_entries(int *n) {')
    reg.append("    static std::vector<pkk::KernelEntry> all = [] {")
    reg.append("        std::vector<pkk::KernelEntry> v;")
    reg.append("        int k = 0;")
    reg.append("        const pkk::KernelEntry *e = nullptr;")
    for grp, _ in tus:
        reg.append("        e = pk_gen_%s(&k);" % grp)
        reg.append("        v.insert(v.end(), e, e + k);")
    reg.append("        return v;")
    reg.append("    }();")
    reg.append("    *n = (int)all.size();")
    reg.append("    return all.data();")
    reg.append("}")
    _write_if_changed(os.path.join(GEN, "registry_gen.cpp"), "\n".join(reg) + "\n")
    return tus


def _write_if_changed(path, text):
    if os.path.exists(path):
        with open(path) as f:
            if f.read() == text:
                return
    with open(path, "w") as f:
        f.write(text)


_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|TotalSGPRs|ScratchSize \[bytes/lane\]|"
                     r"LDS Size \[bytes/block\]|Occupancy \[waves/SIMD\]):\s*(\S+)")


def parse_remarks(text):
    res, cur = {}, None
    for m in _REMARK.finditer(text):
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = val
            res[cur] = {}
        elif cur is not None:
            res[cur][key] = int(val)
    return res


def _compile(src, obj, device):
    cmd = [HIPCC] + COMMON + (DEVICE if device else []) + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, p.stderr[-6000:]))
    return p.stderr


def build(jobs: int = 0, verbose: bool = True) -> str:
    t0 = time.time()
    os.makedirs(BUILD, exist_ok=True)
    tus = generate()
    jobs = jobs or min(16, os.cpu_count() or 4)
    resources = {}
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {}
        for grp, path in tus:
            obj = os.path.join(BUILD, grp + ".o")
            futs[ex.submit(_compile, path, obj, True)] = obj
        for src in HOST_SOURCES:
            obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
            futs[ex.submit(_compile, os.path.join(CSRC, src), obj, False)] = obj
        for src in DEVICE_SOURCES:
            obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
            futs[ex.submit(_compile, os.path.join(CSRC, src), obj, True)] = obj
        futs[ex.submit(_compile, os.path.join(GEN, "registry_gen.cpp"),
                       os.path.join(BUILD, "registry_gen.o"), False)] = os.path.join(BUILD, "registry_gen.o")
        for f in cf.as_completed(futs):
            resources.update(parse_remarks(f.result()))
            objs.append(futs[f])
    names = [name for _, name, _, _ in instances()]
    missing = [n for n in names if n not in resources]
    if missing:
        raise RuntimeError("no resource report for %d kernels, e.g. %s" % (len(missing), missing[:3]))
    lines = ["// generated by build.py from the compiler's kernel-resource-usage report", "",
             "struct pk_gen_resource { const char *name; int vgpr, agpr, sgpr, scratch, lds, occupancy; };",
             "static const pk_gen_resource table[] = {"]
    for n in names:
        r = resources[n]
        lines.append('    {"%s", %d, %d, %d, %d, %d, %d},' % (
            n, r.get("VGPRs", 0), r.get("AGPRs", 0), r.get("TotalSGPRs", 0),
            r.get("ScratchSize [bytes/lane]", 0), r.get("LDS Size [bytes/block]", 0),
            r.get("Occupancy [waves/SIMD]", 0)))
    lines += ["};", 'extern "C" const pk_gen_resource *pk_gen_resources(int *n) {',
              "    *n = (int)(sizeof table / sizeof table[0]);", "    return table;", "}"]
    res_src = os.path.join(GEN, "resources_gen.cpp")
    _write_if_changed(res_src, "\n".join(lines) + "\n")
    res_obj = os.path.join(BUILD, "resources_gen.o")
    _compile(res_src, res_obj, False)
    objs.append(res_obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + sorted(objs)
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stderr[-4000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built %s (%d kernels) in %.1fs" % (LIB, len(names), time.time() - t0), file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
