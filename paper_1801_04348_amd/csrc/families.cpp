// The matmul code fragments the comprehensive optimization runs on, with
// their evaluation functions (Section 3.3) and strategies (Section 3.4).
//
// Machine parameters (Section 3.2), read from hipDeviceProp_t at load time:
//   Z  LDS bytes a workgroup may allocate          (sharedMemPerBlock)
//   V  32-bit registers a workgroup may allocate   (regsPerBlock)
//   T  work-items per workgroup                    (maxThreadsPerBlock)
// Resource counters, in gamma order (shared memory first, then registers, as
// the counter order under which Algorithm 2 yields the systems printed for
// Fig. 6 and Fig. 7), then threads:
//   r_Z  LDS bytes of the workgroup: a polynomial in the program parameters,
//        from the kernel's LDS layout
//   r_V  registers of the workgroup: a table symbol per program (variant),
//        the compiled instance's unified VGPR allocation times its lanes
//   r_T  work-items of the workgroup
//
// VALU family (Section 2, Fig. 4 generalised), program parameters bx (threads
// along N, the paper's ub1), by (threads along M, the paper's B0), s (outputs
// per thread), K tile bk = by as in the paper.  Strategies, omega order:
//   gran  (source; sigma = {r_Z, r_V}) one output per thread, decision (3b)
//   nolds (source; sigma = {r_Z, r_V}) no LDS caching, decision (4b); the
//         direct program also drops the LDS staging registers
// The register-pressure strategy (1) of the experiments has no counterpart:
// the compiler already fits each instance's registers to its launch bounds.
//
// 2-D VALU family (Fig. 4's kernel generalised): program parameters bx, by,
// s (outputs per work-item along N), sy (along M) and bk, the K extent of the
// LDS tiles, free of by; a workgroup owns a (by sy) x (bx s) tile.  LDS bytes
// e (by sy (bk + 1) + bk bx s).  Strategy, omega order:
//   gran  (source; sigma = {r_Z, r_V}) one output per work-item (s = sy = 1)
// The domain holds the 2-D points only (s, sy in {2, 4}, workgroups of one to
// four wavefronts, bk in {16, 32}); one output per work-item in both
// directions is the VALU family's program.
//
// Transposition family (Section 5.2, Fig. 7): program parameters bx (the
// paper's B1, work-items along the columns of A), by (B0), s (elements per
// work-item); strategies gran and nolds as in the VALU family.  LDS bytes of
// the cached program: 4 * (by * s) * (bx + 1) -- one padded tile (the paper's
// program caches a and c separately, 2 s B0 B1 words).
//
// Matrix-addition family (Section 1, Fig. 2): program parameters bx (B1), by
// (B0), s (elements per work-item); counters, in gamma order, r_V and r_T
// only (the two machine parameters of Fig. 2); strategy gran (sigma = {r_V}).
//
// 1D Jacobi family (Section 5, Fig. 6): program parameters B (work-items per
// workgroup, stored as bx) and s (points per work-item); strategies gran and
// nolds as in the VALU family.  LDS bytes of the cached program:
// 4 * (s * B + 2) -- the tile's inputs with one halo point on each side (the
// paper's program caches inputs and outputs, 2 s B + 2 words).
//
// Polynomial-division family (Section 5, Fig. 8): program parameters B and
// s as the 1D Jacobi family, same strategies.  LDS bytes of the cached
// program: 4 * (2 * s * B + 1) -- the tile's a and b values and the leading
// coefficient (the paper's program, 2 s B + 2 words).
//
// MFMA family, program parameters bm, bn (output tile), bk (K tile), wm, wn
// (wavefront grid).  Strategy:
//   single (source; sigma = {r_Z, r_V}) one LDS stage instead of two (also no
//          registers holding the next tile while the current one is used)
#include <algorithm>
#include <stdexcept>

#include "pk_internal.hpp"

namespace pk {

namespace {

struct MfmaPoint {
    int bm, bn, bk, wm, wn;
};

// Program-parameter domains.  VALU: {4, 8, 16, 32}^2 x {1, 2, 4, 8}.
const int kValuB[] = {4, 8, 16, 32};
const int kValuS[] = {1, 2, 4, 8};

// 2-D VALU: (bx, by) with one to four wavefronts, s and sy in {2, 4}, bk in {16, 32}
const int kValu2S[] = {2, 4};
const int kValu2Bk[] = {16, 32};

const int kMaBx[] = {64, 128, 256};
const int kMaBy[] = {1, 2, 4};
const int kMaS[] = {1, 2, 4, 8};
const int kJaB[] = {16, 32, 64, 128, 256, 512, 1024};
const int kJaS[] = {1, 2, 4, 8};
const int kTrBx[] = {16, 32, 64};
const int kTrBy[] = {4, 8, 16, 32};
const int kTrS[] = {1, 2, 4, 8};

const MfmaPoint kMfmaF32[] = {
    {64, 64, 32, 2, 2},   {128, 64, 32, 2, 2},  {64, 128, 32, 2, 2},  {128, 128, 32, 2, 2},
    {256, 128, 32, 4, 2}, {128, 256, 32, 2, 4}, {256, 256, 32, 4, 4}, {256, 128, 32, 2, 2},
    {128, 256, 32, 2, 2}, {256, 128, 16, 4, 2}, {128, 256, 16, 2, 4},
};
const MfmaPoint kMfmaI32[] = {
    {64, 64, 32, 2, 2}, {128, 64, 32, 2, 2}, {64, 128, 32, 2, 2}, {64, 64, 64, 2, 2},
};
const MfmaPoint kMfmaBf16[] = {
    {64, 64, 64, 2, 2},   {128, 64, 64, 2, 2},  {64, 128, 64, 2, 2},  {128, 128, 64, 2, 2},
    {256, 128, 64, 4, 2}, {128, 256, 64, 2, 4}, {256, 256, 64, 4, 4}, {256, 128, 32, 2, 2},
    {128, 256, 32, 2, 2}, {256, 128, 64, 2, 2}, {128, 256, 64, 2, 2},
};

struct Syms {
    int Z, V, T;
};

// Machine symbols Z (LDS bytes), V (registers) and T (work-items) per
// workgroup; a family that uses no LDS has no Z.
Syms add_machine(Family &f, bool lds = true) {
    const int first = lds ? 0 : 1;
    const char *names[] = {"Z", "V", "T"};
    for (int i = first; i < 3; ++i) {
        f.sym_names.push_back(names[i]);
        f.sym_kind.push_back(SYM_MACHINE);
        f.lo.push_back(0);
        f.hi.push_back(INT64_MAX / 4);
    }
    return lds ? Syms{0, 1, 2} : Syms{-1, 0, 1};
}

int add_sym(Family &f, const char *name, int kind) {
    f.sym_names.push_back(name);
    f.sym_kind.push_back(kind);
    f.lo.push_back(0);
    f.hi.push_back(INT64_MAX / 4);
    return (int)f.sym_names.size() - 1;
}

Poly P(int64_t c) { return Poly::constant(c); }
Poly S(int id) { return Poly::symbol(id); }

int64_t table_regs(int family, int variant, int dtype, const std::vector<int64_t> &pt, int wave) {
    const KernelEntry *e = find_instance(family, variant, dtype, pt);
    if (!e) return missing_table_value;
    const KernelResources *r = resources_of(e->name);
    if (!r) return missing_table_value;
    int64_t v = regs_per_block(*r, e->threads, wave);
    // an MFMA program runs as its element-load twin on unaligned rows, and in
    // its split form when split along K: the program needs the largest of
    // the register allocations
    for (const KernelEntry *t : {element_twin(*e), split_twin(*e)})
        if (t)
            if (const KernelResources *rt = resources_of(t->name))
                v = std::max(v, regs_per_block(*rt, t->threads, wave));
    return v;
}

}  // namespace

// gfx950: per-lane allocation = align(align(VGPRs, 4) + AGPRs, 8); a
// workgroup occupies whole wavefronts.
int64_t regs_per_block(const KernelResources &r, int threads, int wave) {
    int64_t v = ((int64_t)r.vgpr + 3) / 4 * 4 + r.agpr;
    v = (v + 7) / 8 * 8;
    int64_t waves = (threads + wave - 1) / wave;
    return v * wave * waves;
}

Family matmul_family(int family, int dtype) {
    Family f;
    Syms m = add_machine(f, family != PK_FAMILY_MADD);
    if (family == PK_FAMILY_VALU) {
        if (dtype != PK_F32 && dtype != PK_I32) throw std::runtime_error("VALU family: f32 and i32 only");
        const int bx = add_sym(f, "bx", SYM_PROGRAM), by = add_sym(f, "by", SYM_PROGRAM),
                  s = add_sym(f, "s", SYM_PROGRAM);
        const int rho_t = add_sym(f, "rho_tiled", SYM_TABLE), rho_t1 = add_sym(f, "rho_tiled_s1", SYM_TABLE),
                  rho_d = add_sym(f, "rho_direct", SYM_TABLE), rho_d1 = add_sym(f, "rho_direct_s1", SYM_TABLE);
        const int64_t es = 4;  // element bytes (float32 and int32)
        f.point_syms = {bx, by, s};
        for (int x : kValuB)
            for (int y : kValuB)
                for (int z : kValuS) f.points.push_back({x, y, z});
        // LDS bytes: A tile by x (bk + 1) and B tile bk x (bx * s), bk = by
        const Poly lds_full = P(es) * (S(by) * (S(by) + P(1)) + S(by) * S(bx) * S(s));
        const Poly lds_g1 = P(es) * (S(by) * (S(by) + P(1)) + S(by) * S(bx));
        CounterDef rz{"r_Z", false, m.Z, nullptr};
        rz.value = [=](uint32_t ap) {
            if (ap & PK_VALU_NOLDS) return P(0);
            if (ap & PK_VALU_GRAN) return lds_g1;
            return lds_full;
        };
        CounterDef rv{"r_V", false, m.V, nullptr};
        rv.value = [=](uint32_t ap) {
            const bool g = ap & PK_VALU_GRAN, d = ap & PK_VALU_NOLDS;
            return S(d ? (g ? rho_d1 : rho_d) : (g ? rho_t1 : rho_t));
        };
        CounterDef rt{"r_T", false, m.T, nullptr};
        rt.value = [=](uint32_t) { return S(bx) * S(by); };
        f.counters = {rz, rv, rt};
        f.strategies = {StrategyDef{"gran", false, 0b011u}, StrategyDef{"nolds", false, 0b011u}};
        f.table = [=](int sym, const std::vector<int64_t> &pt) -> int64_t {
            int variant = 0;
            if (sym == rho_t1 || sym == rho_d1) variant |= PK_VALU_GRAN;
            if (sym == rho_d || sym == rho_d1) variant |= PK_VALU_NOLDS;
            return table_regs(PK_FAMILY_VALU, variant, dtype, pt, 64);
        };
        return f;
    }
    if (family == PK_FAMILY_VALU2) {
        if (dtype != PK_F32 && dtype != PK_I32) throw std::runtime_error("2-D VALU family: f32 and i32 only");
        const int bx = add_sym(f, "bx", SYM_PROGRAM), by = add_sym(f, "by", SYM_PROGRAM),
                  s = add_sym(f, "s", SYM_PROGRAM), sy = add_sym(f, "sy", SYM_PROGRAM),
                  bk = add_sym(f, "bk", SYM_PROGRAM);
        const int rho_t = add_sym(f, "rho_tiled", SYM_TABLE), rho_t1 = add_sym(f, "rho_tiled_s1", SYM_TABLE);
        const int64_t es = 4;
        f.point_syms = {bx, by, s, sy, bk};
        for (int x : kValuB)
            for (int y : kValuB) {
                if (x * y < 64 || x * y > 256) continue;
                for (int z : kValu2S)
                    for (int zy : kValu2S)
                        for (int k : kValu2Bk) f.points.push_back({x, y, z, zy, k});
            }
        // LDS bytes: A tile (by sy) x (bk + 4) and B tile bk x (bx s)
        const Poly lds_full = P(es) * (S(by) * S(sy) * (S(bk) + P(4)) + S(bk) * S(bx) * S(s));
        const Poly lds_g1 = P(es) * (S(by) * (S(bk) + P(4)) + S(bk) * S(bx));
        CounterDef rz{"r_Z", false, m.Z, nullptr};
        rz.value = [=](uint32_t ap) { return (ap & PK_VALU_GRAN) ? lds_g1 : lds_full; };
        CounterDef rv{"r_V", false, m.V, nullptr};
        rv.value = [=](uint32_t ap) { return S((ap & PK_VALU_GRAN) ? rho_t1 : rho_t); };
        CounterDef rt{"r_T", false, m.T, nullptr};
        rt.value = [=](uint32_t) { return S(bx) * S(by); };
        f.counters = {rz, rv, rt};
        f.strategies = {StrategyDef{"gran", false, 0b011u}};
        f.table = [=](int sym, const std::vector<int64_t> &pt) -> int64_t {
            return table_regs(PK_FAMILY_VALU2, sym == rho_t1 ? PK_VALU_GRAN : 0, dtype, pt, 64);
        };
        return f;
    }
    if (family == PK_FAMILY_JACOBI || family == PK_FAMILY_POLYDIV) {
        const bool pd = family == PK_FAMILY_POLYDIV;
        if (pd && dtype != PK_I32) throw std::runtime_error("polynomial division: 32-bit residues (i32) only");
        if (dtype != PK_F32 && dtype != PK_I32) throw std::runtime_error("1D Jacobi: f32 and i32 only");
        const int b = add_sym(f, "B", SYM_PROGRAM), s = add_sym(f, "s", SYM_PROGRAM);
        const int rho_t = add_sym(f, "rho_tiled", SYM_TABLE), rho_t1 = add_sym(f, "rho_tiled_s1", SYM_TABLE),
                  rho_d = add_sym(f, "rho_direct", SYM_TABLE), rho_d1 = add_sym(f, "rho_direct_s1", SYM_TABLE);
        f.point_syms = {b, s};
        for (int x : kJaB)
            for (int z : kJaS) f.points.push_back({x, z});
        const Poly lds_full = pd ? P(8) * S(s) * S(b) + P(4) : P(4) * (S(s) * S(b) + P(2));
        const Poly lds_g1 = pd ? P(8) * S(b) + P(4) : P(4) * (S(b) + P(2));
        CounterDef rz{"r_Z", false, m.Z, nullptr};
        rz.value = [=](uint32_t ap) {
            if (ap & PK_VALU_NOLDS) return P(0);
            if (ap & PK_VALU_GRAN) return lds_g1;
            return lds_full;
        };
        CounterDef rv{"r_V", false, m.V, nullptr};
        rv.value = [=](uint32_t ap) {
            const bool g = ap & PK_VALU_GRAN, d = ap & PK_VALU_NOLDS;
            return S(d ? (g ? rho_d1 : rho_d) : (g ? rho_t1 : rho_t));
        };
        CounterDef rt{"r_T", false, m.T, nullptr};
        rt.value = [=](uint32_t) { return S(b); };
        f.counters = {rz, rv, rt};
        f.strategies = {StrategyDef{"gran", false, 0b011u}, StrategyDef{"nolds", false, 0b011u}};
        f.table = [=](int sym, const std::vector<int64_t> &pt) -> int64_t {
            int variant = 0;
            if (sym == rho_t1 || sym == rho_d1) variant |= PK_VALU_GRAN;
            if (sym == rho_d || sym == rho_d1) variant |= PK_VALU_NOLDS;
            return table_regs(family, variant, dtype, pt, 64);
        };
        return f;
    }
    if (family == PK_FAMILY_MADD) {
        if (dtype != PK_F32 && dtype != PK_I32) throw std::runtime_error("matrix addition: f32 and i32 only");
        const int bx = add_sym(f, "bx", SYM_PROGRAM), by = add_sym(f, "by", SYM_PROGRAM),
                  s = add_sym(f, "s", SYM_PROGRAM);
        const int rho = add_sym(f, "rho", SYM_TABLE), rho1 = add_sym(f, "rho_s1", SYM_TABLE);
        f.point_syms = {bx, by, s};
        for (int x : kMaBx)
            for (int y : kMaBy)
                for (int z : kMaS) f.points.push_back({x, y, z});
        CounterDef rv{"r_V", false, m.V, nullptr};
        rv.value = [=](uint32_t ap) { return S((ap & PK_VALU_GRAN) ? rho1 : rho); };
        CounterDef rt{"r_T", false, m.T, nullptr};
        rt.value = [=](uint32_t) { return S(bx) * S(by); };
        f.counters = {rv, rt};
        f.strategies = {StrategyDef{"gran", false, 0b01u}};
        f.table = [=](int sym, const std::vector<int64_t> &pt) -> int64_t {
            return table_regs(PK_FAMILY_MADD, sym == rho1 ? PK_VALU_GRAN : 0, dtype, pt, 64);
        };
        return f;
    }
    if (family == PK_FAMILY_TRANSPOSE) {
        if (dtype != PK_F32 && dtype != PK_I32) throw std::runtime_error("transposition: 4-byte elements only");
        const int bx = add_sym(f, "bx", SYM_PROGRAM), by = add_sym(f, "by", SYM_PROGRAM),
                  s = add_sym(f, "s", SYM_PROGRAM);
        const int rho_t = add_sym(f, "rho_tiled", SYM_TABLE), rho_t1 = add_sym(f, "rho_tiled_s1", SYM_TABLE),
                  rho_d = add_sym(f, "rho_direct", SYM_TABLE), rho_d1 = add_sym(f, "rho_direct_s1", SYM_TABLE);
        f.point_syms = {bx, by, s};
        for (int x : kTrBx)
            for (int y : kTrBy)
                for (int z : kTrS) f.points.push_back({x, y, z});
        const Poly lds_full = P(4) * S(by) * S(s) * (S(bx) + P(1));
        const Poly lds_g1 = P(4) * S(by) * (S(bx) + P(1));
        CounterDef rz{"r_Z", false, m.Z, nullptr};
        rz.value = [=](uint32_t ap) {
            if (ap & PK_VALU_NOLDS) return P(0);
            if (ap & PK_VALU_GRAN) return lds_g1;
            return lds_full;
        };
        CounterDef rv{"r_V", false, m.V, nullptr};
        rv.value = [=](uint32_t ap) {
            const bool g = ap & PK_VALU_GRAN, d = ap & PK_VALU_NOLDS;
            return S(d ? (g ? rho_d1 : rho_d) : (g ? rho_t1 : rho_t));
        };
        CounterDef rt{"r_T", false, m.T, nullptr};
        rt.value = [=](uint32_t) { return S(bx) * S(by); };
        f.counters = {rz, rv, rt};
        f.strategies = {StrategyDef{"gran", false, 0b011u}, StrategyDef{"nolds", false, 0b011u}};
        f.table = [=](int sym, const std::vector<int64_t> &pt) -> int64_t {
            int variant = 0;
            if (sym == rho_t1 || sym == rho_d1) variant |= PK_VALU_GRAN;
            if (sym == rho_d || sym == rho_d1) variant |= PK_VALU_NOLDS;
            return table_regs(PK_FAMILY_TRANSPOSE, variant, PK_F32, pt, 64);
        };
        return f;
    }
    if (family == PK_FAMILY_MFMA) {
        if (dtype != PK_F32 && dtype != PK_BF16 && dtype != PK_I32)
            throw std::runtime_error("MFMA family: f32, bf16 and i32 only");
        const int bm = add_sym(f, "bm", SYM_PROGRAM), bn = add_sym(f, "bn", SYM_PROGRAM),
                  bk = add_sym(f, "bk", SYM_PROGRAM), wm = add_sym(f, "wm", SYM_PROGRAM),
                  wn = add_sym(f, "wn", SYM_PROGRAM);
        const int rho2 = add_sym(f, "rho_two_stage", SYM_TABLE), rho1 = add_sym(f, "rho_one_stage", SYM_TABLE);
        f.point_syms = {bm, bn, bk, wm, wn};
        if (dtype == PK_F32)
            for (const auto &p : kMfmaF32) f.points.push_back({p.bm, p.bn, p.bk, p.wm, p.wn});
        else if (dtype == PK_I32)
            for (const auto &p : kMfmaI32) f.points.push_back({p.bm, p.bn, p.bk, p.wm, p.wn});
        else
            for (const auto &p : kMfmaBf16) f.points.push_back({p.bm, p.bn, p.bk, p.wm, p.wn});
        // one stage: f32  4 * (bm * (bk + 4) + bk * (bn + 4))
        //            bf16 2 * (bm * (bk + 8) + bk * (bn + 32))
        //            i32  4 * (bm + bn) * (bk + 16)  (four one-byte digit planes
        //                 per operand, rows bk + 16 bytes apart)
        Poly stage = dtype == PK_F32   ? P(4) * (S(bm) * (S(bk) + P(4)) + S(bk) * (S(bn) + P(4)))
                     : dtype == PK_I32 ? P(4) * (S(bm) + S(bn)) * (S(bk) + P(16))
                                       : P(2) * (S(bm) * (S(bk) + P(8)) + S(bk) * (S(bn) + P(32)));
        CounterDef rz{"r_Z", false, m.Z, nullptr};
        rz.value = [=](uint32_t ap) { return (ap & PK_MFMA_SINGLE) ? stage : P(2) * stage; };
        CounterDef rv{"r_V", false, m.V, nullptr};
        rv.value = [=](uint32_t ap) { return S((ap & PK_MFMA_SINGLE) ? rho1 : rho2); };
        CounterDef rt{"r_T", false, m.T, nullptr};
        rt.value = [=](uint32_t) { return P(64) * S(wm) * S(wn); };
        f.counters = {rz, rv, rt};
        f.strategies = {StrategyDef{"single", false, 0b011u}};
        f.table = [=](int sym, const std::vector<int64_t> &pt) -> int64_t {
            return table_regs(PK_FAMILY_MFMA, sym == rho1 ? PK_MFMA_SINGLE : 0, dtype, pt, 64);
        };
        return f;
    }
    throw std::runtime_error("unknown family");
}

bool params_point(int family, const pk_params &p, std::vector<int64_t> *pt) {
    if (family == PK_FAMILY_JACOBI || family == PK_FAMILY_POLYDIV) {
        if (p.by != 0 && p.by != 1) return false;
        *pt = {p.bx, p.s};
        return true;
    }
    if (family == PK_FAMILY_TRANSPOSE || family == PK_FAMILY_MADD) {
        *pt = {p.bx, p.by, p.s};
        return true;
    }
    if (family == PK_FAMILY_VALU) {
        if (p.bk != 0 && p.bk != p.by) return false;  // the paper's K tile: bk = by
        if (p.sy > 1) return false;                     // one output row per work-item
        *pt = {p.bx, p.by, p.s};
        return true;
    }
    if (family == PK_FAMILY_VALU2) {
        *pt = {p.bx, p.by, p.s, p.sy, p.bk};
        return true;
    }
    if (family == PK_FAMILY_MFMA) {
        *pt = {p.bm, p.bn, p.bk, p.wm, p.wn};
        return true;
    }
    return false;
}

void point_params(int family, const std::vector<int64_t> &pt, pk_params *p) {
    p->family = family;
    p->bx = p->by = p->s = p->bk = p->bm = p->bn = p->wm = p->wn = p->sy = p->ks = 0;
    if (family == PK_FAMILY_VALU2) {
        p->bx = (int32_t)pt[0];
        p->by = (int32_t)pt[1];
        p->s = (int32_t)pt[2];
        p->sy = (int32_t)pt[3];
        p->bk = (int32_t)pt[4];
        return;
    }
    if (family == PK_FAMILY_JACOBI || family == PK_FAMILY_POLYDIV) {
        p->bx = (int32_t)pt[0];
        p->by = 1;
        p->s = (int32_t)pt[1];
        return;
    }
    if (family == PK_FAMILY_VALU || family == PK_FAMILY_TRANSPOSE || family == PK_FAMILY_MADD) {
        p->bx = (int32_t)pt[0];
        p->by = (int32_t)pt[1];
        p->s = (int32_t)pt[2];
        p->bk = family == PK_FAMILY_VALU ? (int32_t)pt[1] : 0;
    } else {
        p->bm = (int32_t)pt[0];
        p->bn = (int32_t)pt[1];
        p->bk = (int32_t)pt[2];
        p->wm = (int32_t)pt[3];
        p->wn = (int32_t)pt[4];
    }
}

std::vector<int64_t> machine_values(const Family &fam, const pk_machine &m) {
    std::vector<int64_t> v(fam.sym_names.size(), 0);
    if (fam.sym("Z") >= 0) v[fam.sym("Z")] = m.lds_block;
    v[fam.sym("V")] = m.regs_block;
    v[fam.sym("T")] = m.max_threads_block;
    return v;
}

bool variant_fits(const Family &fam, uint32_t variant, const std::vector<int64_t> &pt,
                  const std::vector<int64_t> &machine_vals) {
    System sys;
    for (const auto &c : fam.counters) {
        if (c.performance) continue;
        sys.push_back(Constraint{c.value(variant), Poly::symbol(c.limit), false});
    }
    return system_holds(fam, sys, pt, machine_vals);
}

const KernelEntry *find_instance(int family, int variant, int dtype, const std::vector<int64_t> &pt) {
    // the program of a variant: VALU granularity reduction runs the s = 1
    // instance; no-LDS runs the direct kernel; MFMA single runs one stage
    int kind = 0;
    std::vector<int64_t> q = pt;
    if (family == PK_FAMILY_TRANSPOSE) dtype = PK_F32;  // a bit copy: one instance serves every 4-byte type
    if (family == PK_FAMILY_JACOBI || family == PK_FAMILY_POLYDIV) {
        const int64_t s = (variant & PK_VALU_GRAN) ? 1 : pt[1];
        for (const auto &e : registry())
            if (e.family == family && e.dtype == dtype && e.variant == (variant & PK_VALU_NOLDS) && e.bx == pt[0] &&
                e.s == s)
                return &e;
        return nullptr;
    }
    if (family == PK_FAMILY_VALU2) {
        // granularity reduction runs the one-output program of the same
        // workgroup and K extent
        const int64_t sx = (variant & PK_VALU_GRAN) ? 1 : pt[2], sy = (variant & PK_VALU_GRAN) ? 1 : pt[3];
        for (const auto &e : registry())
            if (e.family == family && e.dtype == dtype && e.variant == 0 && e.bx == pt[0] && e.by == pt[1] &&
                e.s == sx && e.sy == sy && e.bk == pt[4])
                return &e;
        return nullptr;
    }
    if (family == PK_FAMILY_VALU || family == PK_FAMILY_TRANSPOSE || family == PK_FAMILY_MADD) {
        if (variant & PK_VALU_GRAN) q[2] = 1;
        kind = variant & PK_VALU_NOLDS;
    } else {
        // grouped instances come as a wide kernel and its element-load twin
        kind = variant & (PK_MFMA_SINGLE | PK_MFMA_GROUPED | ((variant & PK_MFMA_GROUPED) ? PK_MFMA_ELEMENT : 0));
    }
    for (const auto &e : registry()) {
        if (e.family != family || e.dtype != dtype || e.variant != kind) continue;
        if (family == PK_FAMILY_VALU || family == PK_FAMILY_TRANSPOSE || family == PK_FAMILY_MADD) {
            if (e.bx == q[0] && e.by == q[1] && e.s == q[2]) return &e;
        } else {
            if (e.bm == q[0] && e.bn == q[1] && e.bk == q[2] && e.wm == q[3] && e.wn == q[4]) return &e;
        }
    }
    return nullptr;
}

const KernelEntry *find_polydiv_fused(int variant, int64_t bx, int64_t s) {
    const int v = variant & (PK_POLYDIV_FUSED | PK_POLYDIV_WIDE);
    for (const auto &e : registry())
        if (e.family == PK_FAMILY_POLYDIV && e.variant == v && e.bx == bx && e.s == s) return &e;
    return nullptr;
}

const KernelEntry *element_twin(const KernelEntry &e) {
    if (e.family != PK_FAMILY_MFMA || (e.variant & (PK_MFMA_GROUPED | PK_MFMA_ELEMENT))) return nullptr;
    for (const auto &t : registry())
        if (t.family == PK_FAMILY_MFMA && t.dtype == e.dtype && t.variant == (e.variant | PK_MFMA_ELEMENT) &&
            t.bm == e.bm && t.bn == e.bn && t.bk == e.bk && t.wm == e.wm && t.wn == e.wn)
            return &t;
    return nullptr;
}

const KernelEntry *split_twin(const KernelEntry &e) {
    if (e.family != PK_FAMILY_MFMA || (e.variant & (PK_MFMA_GROUPED | PK_MFMA_ELEMENT | PK_MFMA_SPLIT))) return nullptr;
    for (const auto &t : registry())
        if (t.family == PK_FAMILY_MFMA && t.dtype == e.dtype && t.variant == (e.variant | PK_MFMA_SPLIT) &&
            t.bm == e.bm && t.bn == e.bn && t.bk == e.bk && t.wm == e.wm && t.wn == e.wn)
            return &t;
    return nullptr;
}

const KernelEntry *find_jacobi_fused(int dtype, int64_t bx, int64_t s) {
    for (const auto &e : registry())
        if (e.family == PK_FAMILY_JACOBI && e.variant == PK_JACOBI_FUSED && e.dtype == dtype && e.bx == bx && e.s == s)
            return &e;
    return nullptr;
}

}  // namespace pk
