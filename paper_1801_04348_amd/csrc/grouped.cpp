// Many independent products in one persistent launch.
//
// A plan fixes, once, everything a grouped launch needs: for every product its
// program (MFMA point and LDS-stage count), its descriptor (pointers, leading
// dimensions, sizes, whether rows are aligned for the wide loads, first global
// tile index, program index) and a tile -> product map.
//
// Kernels.  A uniform grouped kernel runs one tile program for every product;
// a mixed grouped kernel runs, per product, one of the programs kMixedTile
// (64x64, 128x64, 64x128 and 128x128 output tiles of four wavefronts, one
// blockDim), with one LDS allocation sized for the largest of them.  A plan is
// one launch whenever its products' programs are all one program or all
// programs of the mixed kernel with one stage count.
//
// Choice of programs (per_group_or_null NULL):
//   CASE        per product, the program of least estimated compute-unit time
//               (product_cost: the tiles' arithmetic at the residency the
//               launch's kernel reaches, plus each tile's opening loads and
//               closing stores, hidden only by the other resident
//               workgroups); the kernel -- each uniform program that fits
//               every product, each mixed kernel -- of least total estimate
//               wins.
//   EXHAUSTIVE  the auto-tuner: a plan of every uniform program and stage
//               count whose case-table point is feasible for every product,
//               and of each mixed kernel under three per-product rules (the
//               CASE estimate; the largest tile wasting at most 15 % or 35 %
//               of its area on padding), timed on the plan's own operands
//               (one untimed run, median of three); the fastest is kept.
// A product's program is always a point of the case table whose leaf holds
// for the product's shape (the MFMA candidates of pk_select's feasible set).
//
// Tile order.  The launch's products are sorted by estimated cost per tile,
// most expensive first (stable), and the tile list is cut into kXcds
// contiguous ranges of equal estimated cost, one per XCD: workgroup b, which
// the hardware places on XCD b % kXcds, strides over its XCD's range, so a
// product's tiles share one L2 and each range ends with its cheapest tiles.
//
// Descriptors and maps are staged in pinned host memory and copied to the
// device when the plan is created, so running a plan allocates nothing and
// does not synchronise: it can be captured in a HIP graph, and
// pk_grouped_plan_capture does that itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <stdexcept>

#include "grouped.hpp"
#include "pk_internal.hpp"
#include "select.hpp"

using pkk::GroupArgs;
using pkk::GroupDesc;
using pkk::kMixedPrograms;
using pkk::kMixedTile;
using pkk::kXcds;

struct pk_grouped_plan {
    int dtype = 0;
    int device = -1;
    int accumulate = 0;
    pk::GroupedLayout layout;
    void *host = nullptr;  // pinned staging copy
    void *dev = nullptr;   // descriptors, then tile maps
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~pk_grouped_plan() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        if (dev) hipFree(dev);
        if (host) hipHostFree(host);
    }
};

namespace pk {

namespace {

constexpr int kMixedVariant = PK_MFMA_GROUPED | PK_MFMA_MIXED;

// The mixed kernel of a dtype and stage count (0: two stages, PK_MFMA_SINGLE: one).
const KernelEntry *mixed_entry(int dtype, int stage) {
    for (const auto &e : registry())
        if (e.family == PK_FAMILY_MFMA && e.dtype == dtype && e.variant == (kMixedVariant | stage)) return &e;
    return nullptr;
}

// The kernel's own resources fit one workgroup of the bound machine.
bool entry_fits(const pk_machine &m, const KernelEntry &e) {
    if (e.threads > m.max_threads_block || e.lds_bytes > m.lds_block) return false;
    const KernelResources *r = resources_of(e.name);
    return r && regs_per_block(*r, e.threads, m.wave > 0 ? m.wave : 64) <= m.regs_block;
}

// A kernel entry as a product of mixed program `prog` runs in it: the mixed
// kernel's residency, the program's tile.
KernelEntry as_program(const KernelEntry &e, int prog) {
    KernelEntry x = e;
    x.tile_m = kMixedTile[prog][0];
    x.tile_n = kMixedTile[prog][1];
    x.bm = x.tile_m;
    x.bn = x.tile_n;
    return x;
}

bool aligned_rows(int dtype, const void *A, int64_t lda, const void *B, int64_t ldb) {
    return wide_rows(dtype, A, lda, B, ldb);
}

// One product's place in a layout.
struct Assign {
    const KernelEntry *entry = nullptr;  // the launch's kernel
    int prog = 0;                        // mixed kernels: index into kMixedTile
    int tile_m = 0, tile_n = 0;
    double cost = 0.0;                   // estimated compute-unit seconds of its tiles
    pk_params params{};
};

bool live(const GroupedOperands &o, int g) { return o.M[g] > 0 && o.N[g] > 0; }

// Seconds a tile of a persistent grouped launch spends opening (its
// descriptor, then its first K step's operands, loads each waiting on the
// last) and closing (its stores), which nothing in its workgroup overlaps:
// its tiles are a few K steps long and run one after another.  Only the
// other workgroups resident on the compute unit hide it.  Set so that the
// estimate ranks programs as measured on 4096 uneven float32 products of
// 16-512: the 64 x 64 programs of one and two LDS stages, which
// tile_work_seconds rates alike, hold 5 and 4 resident workgroups, and the
// single-stage one runs the products 15 % faster.
constexpr double kTileOpenClose = 5e-6;

// Estimated compute-unit seconds of a product under a grouped program.
double product_cost(const pk_machine &m, const KernelEntry &e, int dtype, int64_t M, int64_t N, int64_t K) {
    const int64_t tiles = ((M + e.tile_m - 1) / e.tile_m) * ((N + e.tile_n - 1) / e.tile_n);
    return tile_work_seconds(m, e, dtype, M, N, K) + (double)tiles * kTileOpenClose / (double)live_blocks_per_cu(m, e);
}

// The grouped kernel form a product runs in: the wide kernel when its rows
// are aligned for 16-byte loads, else the element-load twin (PK_MFMA_ELEMENT).
int form_of(int dtype, const GroupedOperands &o, int g) {
    return o.K[g] > 0 && aligned_rows(dtype, o.A[g], o.lda[g], o.B[g], o.ldb[g]) ? 0 : (int)PK_MFMA_ELEMENT;
}

int check_operands(const GroupedOperands &o) {
    for (int g = 0; g < o.G; ++g) {
        if (o.M[g] < 0 || o.N[g] < 0 || o.K[g] < 0 || o.M[g] > kMaxDim || o.N[g] > kMaxDim || o.K[g] > kMaxDim)
            return fail(PK_ERR_INVALID_ARG, "bad size in product " + std::to_string(g));
        if (!live(o, g)) continue;
        if (!o.C[g] || o.ldc[g] < o.N[g] ||
            (o.K[g] > 0 && (!o.A[g] || !o.B[g] || o.lda[g] < o.K[g] || o.ldb[g] < o.N[g])))
            return fail(PK_ERR_INVALID_ARG, "bad operands in product " + std::to_string(g));
    }
    return PK_OK;
}

pk_params program_params(const std::vector<int64_t> &pt, int stage) {
    pk_params p{};
    point_params(PK_FAMILY_MFMA, pt, &p);
    p.leaf = -1;  // a forced variant: the stage count of the launch
    p.variant = stage;
    return p;
}

// The MFMA points with a leaf of the case table at the bound machine and a
// compiled instance: the MFMA part of pk_select's feasible set, which does not
// depend on the product's shape (the leaves' systems hold or fail on the
// program and machine parameters alone).
struct Feasibility {
    const pk_table::Part *part = nullptr;
    std::vector<char> ok;                               // per point index
    int prog_point[kMixedPrograms] = {-1, -1, -1, -1};  // point index of each mixed program
};

int feasibility(const pk_table *tbl, int dtype, Feasibility *f) {
    f->part = tbl->part(PK_FAMILY_MFMA, dtype);
    if (!f->part || !f->part->supported) return fail(PK_ERR_UNSUPPORTED_DTYPE, "no MFMA family for the dtype");
    const auto &pts = f->part->fam.points;
    for (int p = 0; p < kMixedPrograms; ++p) {
        const std::vector<int64_t> pt = {kMixedTile[p][0], kMixedTile[p][1], pkk::kMixedBk[dtype], 2, 2};
        auto it = std::find(pts.begin(), pts.end(), pt);
        f->prog_point[p] = it == pts.end() ? -1 : (int)(it - pts.begin());
    }
    f->ok.assign(pts.size(), 0);
    bool any = false;
    for (size_t i = 0; i < pts.size(); ++i) {
        const int leaf = f->part->first_leaf[i];
        if (leaf < 0) continue;
        const int variant = (int)f->part->solved.leaves[leaf].applied;
        if (find_instance(PK_FAMILY_MFMA, variant, dtype, pts[i])) f->ok[i] = any = 1;
    }
    if (!any) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no MFMA program fits the machine");
    return PK_OK;
}

// Every live product on the uniform grouped instance of point `pi`, stage `stage`.
bool assign_uniform(const pk_table *tbl, int dtype, const GroupedOperands &o, const Feasibility &f, int pi,
                    int stage, std::vector<Assign> *out) {
    if (!f.ok[pi]) return false;
    const auto &pt = f.part->fam.points[pi];
    const KernelEntry *forms[2] = {find_instance(PK_FAMILY_MFMA, stage | PK_MFMA_GROUPED, dtype, pt),
                                   find_instance(PK_FAMILY_MFMA, stage | PK_MFMA_GROUPED | PK_MFMA_ELEMENT, dtype, pt)};
    out->assign(o.G, Assign{});
    for (int g = 0; g < o.G; ++g) {
        if (!live(o, g)) continue;
        const KernelEntry *e = forms[form_of(dtype, o, g) ? 1 : 0];
        if (!e || !entry_fits(tbl->machine, *e)) return false;
        Assign &a = (*out)[g];
        a.entry = e;
        a.tile_m = e->tile_m;
        a.tile_n = e->tile_n;
        a.cost = product_cost(tbl->machine, *e, dtype, o.M[g], o.N[g], o.K[g]);
        a.params = program_params(pt, stage);
    }
    return true;
}

// Rules of the mixed kernel's per-product choice.
enum MixedRule { RULE_ESTIMATE = 0, RULE_WASTE_15, RULE_WASTE_35 };

bool assign_mixed(const pk_table *tbl, int dtype, const GroupedOperands &o, const Feasibility &f, int stage,
                  int rule, std::vector<Assign> *out) {
    const KernelEntry *forms[2] = {mixed_entry(dtype, stage), mixed_entry(dtype, stage | PK_MFMA_ELEMENT)};
    KernelEntry progs_of[2][kMixedPrograms];
    for (int w = 0; w < 2; ++w)
        if (forms[w])
            for (int p = 0; p < kMixedPrograms; ++p) progs_of[w][p] = as_program(*forms[w], p);
    out->assign(o.G, Assign{});
    for (int g = 0; g < o.G; ++g) {
        if (!live(o, g)) continue;
        const int w = form_of(dtype, o, g) ? 1 : 0;
        const KernelEntry *e = forms[w];
        if (!e || !entry_fits(tbl->machine, *e)) return false;
        const KernelEntry *progs = progs_of[w];
        int best = -1;
        double best_cost = 0.0, cost[kMixedPrograms];
        for (int p = 0; p < kMixedPrograms; ++p) {
            cost[p] = -1.0;
            if (f.prog_point[p] < 0 || !f.ok[f.prog_point[p]]) continue;
            cost[p] = product_cost(tbl->machine, progs[p], dtype, o.M[g], o.N[g], o.K[g]);
            if (best < 0 || cost[p] < best_cost) {
                best = p;
                best_cost = cost[p];
            }
        }
        if (best < 0) return false;
        if (rule != RULE_ESTIMATE) {
            const double limit = rule == RULE_WASTE_15 ? 0.15 : 0.35;
            int pick = -1;
            for (int p = 0; p < kMixedPrograms; ++p) {
                if (cost[p] < 0.0) continue;
                const int64_t bm = kMixedTile[p][0], bn = kMixedTile[p][1];
                const double padded = (double)((o.M[g] + bm - 1) / bm * bm) * (double)((o.N[g] + bn - 1) / bn * bn);
                const double waste = padded / ((double)o.M[g] * (double)o.N[g]) - 1.0;
                if (waste > limit) continue;
                if (pick < 0 || bm * bn > kMixedTile[pick][0] * kMixedTile[pick][1] ||
                    (bm * bn == kMixedTile[pick][0] * kMixedTile[pick][1] && cost[p] < cost[pick]))
                    pick = p;
            }
            if (pick >= 0) best = pick;
        }
        Assign &a = (*out)[g];
        a.entry = e;
        a.prog = best;
        a.tile_m = kMixedTile[best][0];
        a.tile_n = kMixedTile[best][1];
        a.cost = cost[best];
        a.params = program_params(f.part->fam.points[f.prog_point[best]], stage);
    }
    return true;
}

double total_cost(const std::vector<Assign> &as) {
    double t = 0.0;
    for (const auto &a : as) t += a.cost;
    return t;
}

// A mixed assignment whose products all run one program runs that program's
// uniform instance instead (fewer registers, the same arithmetic), when it
// fits.
void prefer_uniform(const pk_table *tbl, int dtype, const GroupedOperands &o, std::vector<Assign> *as) {
    const KernelEntry *mixed = nullptr;
    int prog = -1;
    for (int g = 0; g < o.G; ++g) {
        const Assign &a = (*as)[g];
        if (!a.entry) continue;
        if (!(a.entry->variant & PK_MFMA_MIXED)) return;
        if (prog >= 0 && a.prog != prog) return;
        prog = a.prog;
        mixed = a.entry;
    }
    if (!mixed) return;
    const int stage = mixed->variant & PK_MFMA_SINGLE;
    const std::vector<int64_t> pt = {kMixedTile[prog][0], kMixedTile[prog][1], pkk::kMixedBk[dtype], 2, 2};
    const KernelEntry *forms[2] = {find_instance(PK_FAMILY_MFMA, stage | PK_MFMA_GROUPED, dtype, pt),
                                   find_instance(PK_FAMILY_MFMA, stage | PK_MFMA_GROUPED | PK_MFMA_ELEMENT, dtype, pt)};
    for (int g = 0; g < o.G; ++g) {
        const Assign &a = (*as)[g];
        if (!a.entry) continue;
        const KernelEntry *e = forms[(a.entry->variant & PK_MFMA_ELEMENT) ? 1 : 0];
        if (!e || !entry_fits(tbl->machine, *e)) return;
    }
    for (int g = 0; g < o.G; ++g) {
        Assign &a = (*as)[g];
        if (!a.entry) continue;
        const KernelEntry *e = forms[(a.entry->variant & PK_MFMA_ELEMENT) ? 1 : 0];
        a.entry = e;
        a.prog = 0;
        a.cost = product_cost(tbl->machine, *e, dtype, o.M[g], o.N[g], o.K[g]);
    }
}

// The layout of an assignment: one launch per kernel.
int build_from(const pk_table *tbl, int dtype, const GroupedOperands &o, const std::vector<Assign> &as,
               GroupedLayout *out) {
    GroupedLayout lay;
    lay.chosen.assign(o.G, pk_params{});
    std::map<const KernelEntry *, std::vector<int>> by_entry;
    std::vector<const KernelEntry *> order;  // kernels in order of first use
    for (int g = 0; g < o.G; ++g) {
        if (!as[g].entry) continue;
        lay.chosen[g] = as[g].params;
        auto &v = by_entry[as[g].entry];
        if (v.empty()) order.push_back(as[g].entry);
        v.push_back(g);
    }
    for (const KernelEntry *e : order) {
        std::vector<int> gs = by_entry[e];
        std::vector<int64_t> tiles(o.G, 0);
        // estimated cost of one tile of each product: its K steps' work (the
        // estimate of a one-tile product, the same figure for every product
        // of one program and K) plus one step more for what every tile pays
        // once -- the first step's loads, which nothing overlaps, and the
        // stores of its results.  Without that term tiles of one or two K
        // steps count as nearly free and the XCD that gets them runs last.
        std::vector<double> tile_cost(o.G, 0.0);
        for (int g : gs) {
            const Assign &a = as[g];
            tiles[g] = ((o.M[g] + a.tile_m - 1) / a.tile_m) * ((o.N[g] + a.tile_n - 1) / a.tile_n);
            const KernelEntry pe = (a.entry->variant & PK_MFMA_MIXED) ? as_program(*a.entry, a.prog) : *a.entry;
            const int64_t bk = pe.bk > 0 ? pe.bk : 1;
            const double ks = (double)((std::max<int64_t>(o.K[g], 1) + bk - 1) / bk);
            tile_cost[g] = tile_work_seconds(tbl->machine, pe, dtype, pe.tile_m, pe.tile_n, o.K[g]) * (ks + 1.0) / ks;
        }
        // most expensive tiles first
        std::stable_sort(gs.begin(), gs.end(), [&](int x, int y) { return tile_cost[x] > tile_cost[y]; });
        GroupedLaunch L;
        L.entry = e;
        L.first_desc = (int64_t)lay.descs.size();
        L.first_tile = (int64_t)lay.tmap.size();
        double total = 0.0;
        for (int g : gs) total += tile_cost[g] * (double)tiles[g];
        const bool cost_known = total > 0.0;
        if (!cost_known) {  // no estimate: cut by tile count
            total = 0.0;
            for (int g : gs) total += (double)tiles[g];
        }
        int64_t t = 0;
        double cum = 0.0;
        int bin = 1;
        L.bins[0] = 0;
        for (int g : gs) {
            const Assign &a = as[g];
            GroupDesc d;
            std::memset(&d, 0, sizeof d);
            d.A = o.A[g];
            d.B = o.B[g];
            d.C = o.C[g];
            d.lda = o.lda[g];
            d.ldb = o.ldb[g];
            d.ldc = o.ldc[g];
            d.M = (int32_t)o.M[g];
            d.N = (int32_t)o.N[g];
            d.K = (int32_t)o.K[g];
            d.vec = o.K[g] > 0 && aligned_rows(dtype, o.A[g], o.lda[g], o.B[g], o.ldb[g]) ? 1 : 0;
            d.tile_start = t;
            d.tiles_n = (int32_t)((o.N[g] + a.tile_n - 1) / a.tile_n);
            d.prog = a.prog;
            const int32_t local = (int32_t)(lay.descs.size() - L.first_desc);
            const double per_tile = cost_known ? tile_cost[g] : 1.0;
            for (int64_t i = 0; i < tiles[g]; ++i) {
                // cut before this tile where the cost so far reaches the
                // next bin's share
                while (bin < kXcds && cum >= total * bin / kXcds) L.bins[bin++] = t + i;
                lay.tmap.push_back(local);
                cum += per_tile;
            }
            t += tiles[g];
            lay.descs.push_back(d);
        }
        while (bin <= kXcds) L.bins[bin++] = t;
        L.ndesc = (int64_t)lay.descs.size() - L.first_desc;
        L.total_tiles = t;
        L.grid = std::max<int64_t>(1, std::min<int64_t>(t, (int64_t)tbl->machine.cu_count *
                                                             live_blocks_per_cu(tbl->machine, *e)));
        lay.launches.push_back(L);
    }
    *out = std::move(lay);
    return PK_OK;
}

// The parameters each product was given, resolved; one launch when they are
// all one program or all programs of the mixed kernel with one stage count.
int assign_given(const pk_table *tbl, int dtype, const GroupedOperands &o, const pk_params *per_group,
                 std::vector<Assign> *out) {
    out->assign(o.G, Assign{});
    std::vector<std::vector<int64_t>> pts(o.G);
    std::vector<int> stage(o.G, 0);
    bool all_mixed = true, one_program = true;
    int first = -1;
    for (int g = 0; g < o.G; ++g) {
        if (!live(o, g)) continue;
        pk_params p = per_group[g];
        if (p.family != PK_FAMILY_MFMA) return fail(PK_ERR_UNSUPPORTED_DTYPE, "grouped launches run MFMA programs only");
        pk_params q;
        const KernelEntry *e0 = nullptr;
        int rc = resolve(tbl, &p, dtype, &q, &e0);
        if (rc != PK_OK) return rc;
        params_point(PK_FAMILY_MFMA, q, &pts[g]);
        stage[g] = q.variant & PK_MFMA_SINGLE;
        (*out)[g].params = q;
        if (first < 0) first = g;
        if (pts[g] != pts[first] || stage[g] != stage[first]) one_program = false;
        if (stage[g] != stage[first]) all_mixed = false;
        bool in_mixed = false;
        for (int pr = 0; pr < kMixedPrograms; ++pr)
            if (pts[g] == std::vector<int64_t>{kMixedTile[pr][0], kMixedTile[pr][1], pkk::kMixedBk[dtype], 2, 2}) {
                in_mixed = true;
                (*out)[g].prog = pr;
            }
        if (!in_mixed) all_mixed = false;
    }
    if (first < 0) return PK_OK;
    const KernelEntry *mixed_forms[2] = {nullptr, nullptr};
    bool use_mixed = !one_program && all_mixed;
    if (use_mixed)
        for (int g = 0; g < o.G; ++g) {
            if (!live(o, g)) continue;
            const int w = form_of(dtype, o, g) ? 1 : 0;
            if (!mixed_forms[w]) mixed_forms[w] = mixed_entry(dtype, stage[first] | (w ? PK_MFMA_ELEMENT : 0));
            if (!mixed_forms[w] || !entry_fits(tbl->machine, *mixed_forms[w])) use_mixed = false;
        }
    for (int g = 0; g < o.G; ++g) {
        if (!live(o, g)) continue;
        Assign &a = (*out)[g];
        const int w = form_of(dtype, o, g) ? 1 : 0;
        if (use_mixed) {
            const KernelEntry *mixed = mixed_forms[w];
            a.entry = mixed;
            const KernelEntry x = as_program(*mixed, a.prog);
            a.tile_m = x.tile_m;
            a.tile_n = x.tile_n;
            a.cost = product_cost(tbl->machine, x, dtype, o.M[g], o.N[g], o.K[g]);
            continue;
        }
        const KernelEntry *e =
            find_instance(PK_FAMILY_MFMA, stage[g] | PK_MFMA_GROUPED | (w ? PK_MFMA_ELEMENT : 0), dtype, pts[g]);
        if (!e) return fail(PK_ERR_NOT_INSTANTIATED, "no grouped instance for product " + std::to_string(g));
        a.entry = e;
        a.prog = 0;
        a.tile_m = e->tile_m;
        a.tile_n = e->tile_n;
        a.cost = product_cost(tbl->machine, *e, dtype, o.M[g], o.N[g], o.K[g]);
    }
    return PK_OK;
}

// Every candidate assignment of the auto-tuner (uniform programs, mixed
// kernels under each rule); the CASE choice is the one of least total cost.
int candidate_assignments(const pk_table *tbl, int dtype, const GroupedOperands &o, const Feasibility &f,
                          bool all_rules, std::vector<std::vector<Assign>> *out) {
    out->clear();
    for (int pi = 0; pi < (int)f.part->fam.points.size(); ++pi)
        for (int stage : {0, (int)PK_MFMA_SINGLE}) {
            std::vector<Assign> as;
            if (assign_uniform(tbl, dtype, o, f, pi, stage, &as)) out->push_back(std::move(as));
        }
    for (int stage : {0, (int)PK_MFMA_SINGLE})
        for (int rule : {RULE_ESTIMATE, RULE_WASTE_15, RULE_WASTE_35}) {
            if (!all_rules && rule != RULE_ESTIMATE) continue;
            std::vector<Assign> as;
            if (!assign_mixed(tbl, dtype, o, f, stage, rule, &as)) continue;
            prefer_uniform(tbl, dtype, o, &as);
            out->push_back(std::move(as));
        }
    if (out->empty()) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no grouped kernel fits every product");
    return PK_OK;
}

bool same_assignment(const std::vector<Assign> &x, const std::vector<Assign> &y) {
    for (size_t g = 0; g < x.size(); ++g)
        if (x[g].entry != y[g].entry || x[g].prog != y[g].prog) return false;
    return true;
}

// A layout's bytes on the device, for timing a candidate.
struct DeviceCopy {
    void *dev = nullptr;
    ~DeviceCopy() {
        if (dev) hipFree(dev);
    }
};

int upload(const GroupedLayout &lay, void **dev, void *host_stage) {
    const size_t dbytes = lay.descs.size() * sizeof(GroupDesc);
    if (host_stage) {
        std::memcpy(host_stage, lay.descs.data(), dbytes);
        std::memcpy((char *)host_stage + dbytes, lay.tmap.data(), lay.tmap.size() * sizeof(int32_t));
    }
    hipError_t err = hipMalloc(dev, lay.bytes());
    if (err == hipSuccess && host_stage) err = hipMemcpy(*dev, host_stage, lay.bytes(), hipMemcpyHostToDevice);
    if (err == hipSuccess && !host_stage) {
        err = hipMemcpy(*dev, lay.descs.data(), dbytes, hipMemcpyHostToDevice);
        if (err == hipSuccess && !lay.tmap.empty())
            err = hipMemcpy((char *)*dev + dbytes, lay.tmap.data(), lay.tmap.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice);
    }
    if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("grouped layout upload: ") + hipGetErrorString(err));
    return PK_OK;
}

// seconds per run of a layout: one untimed run, then the median of three
int time_layout(int device, const GroupedLayout &lay, const void *dev, double *secs) {
    hipError_t err = hipSetDevice(device);
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (err == hipSuccess) err = hipStreamCreate(&s);
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    int rc = err == hipSuccess ? grouped_launch(lay, dev, 0, s) : PK_ERR_HIP;
    float t[3] = {0.f, 0.f, 0.f};
    for (int i = 0; i < 3 && rc == PK_OK && err == hipSuccess; ++i) {
        err = hipEventRecord(e0, s);
        if (err == hipSuccess) rc = grouped_launch(lay, dev, 0, s);
        if (err == hipSuccess && rc == PK_OK) err = hipEventRecord(e1, s);
        if (err == hipSuccess && rc == PK_OK) err = hipEventSynchronize(e1);
        if (err == hipSuccess && rc == PK_OK) err = hipEventElapsedTime(&t[i], e0, e1);
    }
    if (s) hipStreamSynchronize(s);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (s) hipStreamDestroy(s);
    if (rc != PK_OK) return rc;
    if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("timing a grouped plan: ") + hipGetErrorString(err));
    std::sort(t, t + 3);
    *secs = 1e-3 * t[1];
    return PK_OK;
}

}  // namespace

int grouped_layout(const pk_table *tbl, int dtype, const GroupedOperands &o, const pk_params *per_group,
                   GroupedLayout *out) {
    int rc = check_operands(o);
    if (rc != PK_OK) return rc;
    std::vector<Assign> as;
    if (per_group) {
        rc = assign_given(tbl, dtype, o, per_group, &as);
        if (rc != PK_OK) return rc;
        return build_from(tbl, dtype, o, as, out);
    }
    Feasibility f;
    rc = feasibility(tbl, dtype, &f);
    if (rc != PK_OK) return rc;
    std::vector<std::vector<Assign>> cands;
    rc = candidate_assignments(tbl, dtype, o, f, false, &cands);
    if (rc != PK_OK) return rc;
    size_t best = 0;
    for (size_t i = 1; i < cands.size(); ++i)
        if (total_cost(cands[i]) < total_cost(cands[best])) best = i;
    return build_from(tbl, dtype, o, cands[best], out);
}

int grouped_launch(const GroupedLayout &lay, const void *dev, int accumulate, hipStream_t stream) {
    const size_t dbytes = lay.descs.size() * sizeof(GroupDesc);
    for (const auto &L : lay.launches) {
        GroupArgs a;
        std::memset(&a, 0, sizeof a);
        a.descs = (const GroupDesc *)dev + L.first_desc;
        a.tile_group = (const int32_t *)((const char *)dev + dbytes) + L.first_tile;
        a.total_tiles = L.total_tiles;
        a.accumulate = accumulate;
        for (int x = 0; x <= kXcds; ++x) a.bin_first[x] = L.bins[x];
        void *kargs[] = {&a};
        hipError_t err = hipLaunchKernel(L.entry->fn, dim3((unsigned)L.grid), dim3((unsigned)L.entry->threads), kargs,
                                         0, stream);
        if (err != hipSuccess)
            return fail(PK_ERR_HIP, std::string("hipLaunchKernel(") + L.entry->name + "): " + hipGetErrorString(err));
    }
    return PK_OK;
}

}  // namespace pk

using namespace pk;

extern "C" {

int pk_grouped_plan_create(const pk_table *tbl, pk_dtype dtype, int32_t G, const int64_t *M, const int64_t *N,
                           const int64_t *K, const void *const *A, const int64_t *lda, const void *const *B,
                           const int64_t *ldb, void *const *C, const int64_t *ldc,
                           const pk_params *per_group_or_null, int policy, int accumulate,
                           pk_grouped_plan **out) {
    if (!tbl || !out || G < 0 || (G > 0 && (!M || !N || !K || !A || !lda || !B || !ldb || !C || !ldc)))
        return fail(PK_ERR_INVALID_ARG, "null argument or negative group count");
    *out = nullptr;
    if (dtype != PK_F32 && dtype != PK_BF16) return fail(PK_ERR_UNSUPPORTED_DTYPE, "grouped products: f32 or bf16");
    if (tbl->device < 0) return fail(PK_ERR_INVALID_ARG, "grouped plans need a table bound to a device");
    if (policy == PK_POLICY_LEARNED)
        return fail(PK_ERR_INVALID_ARG,
                    "grouped plans: policy CASE or EXHAUSTIVE (the cost model predicts single launches, not the "
                    "share of a persistent launch a product takes)");
    if (policy != PK_POLICY_CASE && policy != PK_POLICY_EXHAUSTIVE)
        return fail(PK_ERR_INVALID_ARG, "grouped plans: policy CASE or EXHAUSTIVE");
    if (policy == PK_POLICY_EXHAUSTIVE && accumulate && !per_group_or_null)
        return fail(PK_ERR_INVALID_ARG, "grouped plans: EXHAUSTIVE selection writes C, so not with accumulate");
    try {
        GroupedOperands o;
        o.G = G;
        o.M = M, o.N = N, o.K = K, o.A = A, o.lda = lda, o.B = B, o.ldb = ldb, o.C = C, o.ldc = ldc;
        std::unique_ptr<pk_grouped_plan> plan(new pk_grouped_plan);
        plan->dtype = (int)dtype;
        plan->device = tbl->device;
        plan->accumulate = accumulate ? 1 : 0;
        hipError_t err = hipSetDevice(tbl->device);
        if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(err));
        int rc = PK_OK;
        if (policy == PK_POLICY_EXHAUSTIVE && !per_group_or_null) {
            rc = check_operands(o);
            if (rc != PK_OK) return rc;
            Feasibility f;
            rc = feasibility(tbl, (int)dtype, &f);
            if (rc != PK_OK) return rc;
            std::vector<std::vector<Assign>> cands;
            rc = candidate_assignments(tbl, (int)dtype, o, f, true, &cands);
            if (rc != PK_OK) return rc;
            double best_s = 0.0;
            int best = -1;
            for (size_t i = 0; i < cands.size(); ++i) {
                bool dup = false;
                for (size_t j = 0; j < i && !dup; ++j) dup = same_assignment(cands[i], cands[j]);
                if (dup) continue;
                GroupedLayout lay;
                rc = build_from(tbl, (int)dtype, o, cands[i], &lay);
                if (rc != PK_OK) return rc;
                DeviceCopy dc;
                if (lay.bytes() > 0) {
                    rc = upload(lay, &dc.dev, nullptr);
                    if (rc != PK_OK) return rc;
                }
                double secs = 0.0;
                rc = time_layout(tbl->device, lay, dc.dev, &secs);
                if (rc != PK_OK) return rc;
                if (best < 0 || secs < best_s) {
                    best = (int)i;
                    best_s = secs;
                }
            }
            rc = build_from(tbl, (int)dtype, o, cands[best], &plan->layout);
        } else {
            rc = grouped_layout(tbl, (int)dtype, o, per_group_or_null, &plan->layout);
        }
        if (rc != PK_OK) return rc;
        const size_t bytes = plan->layout.bytes();
        if (bytes > 0) {
            err = hipHostMalloc(&plan->host, bytes, hipHostMallocDefault);
            if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("grouped plan: ") + hipGetErrorString(err));
            rc = upload(plan->layout, &plan->dev, plan->host);
            if (rc != PK_OK) return rc;
        }
        *out = plan.release();
        return PK_OK;
    } catch (const std::exception &ex) {
        return fail(PK_ERR_INVALID_ARG, ex.what());
    }
}

int pk_grouped_plan_run(const pk_grouped_plan *plan, void *hip_stream) {
    if (!plan) return fail(PK_ERR_INVALID_ARG, "null plan");
    return grouped_launch(plan->layout, plan->dev, plan->accumulate, (hipStream_t)hip_stream);
}

int pk_grouped_plan_capture(pk_grouped_plan *plan) {
    if (!plan) return fail(PK_ERR_INVALID_ARG, "null plan");
    if (plan->exec) return PK_OK;
    hipStream_t s;
    hipError_t err = hipSetDevice(plan->device);
    if (err == hipSuccess) err = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("capture stream: ") + hipGetErrorString(err));
    err = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    int rc = PK_OK;
    if (err == hipSuccess) rc = pk_grouped_plan_run(plan, s);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &g);
    hipStreamDestroy(s);
    if (err != hipSuccess || e2 != hipSuccess || rc != PK_OK) {
        if (g) hipGraphDestroy(g);
        return rc != PK_OK ? rc : fail(PK_ERR_HIP, std::string("capture: ") + hipGetErrorString(err != hipSuccess ? err : e2));
    }
    err = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        hipGraphDestroy(g);
        return fail(PK_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(err));
    }
    plan->graph = g;
    return PK_OK;
}

int pk_grouped_plan_replay(const pk_grouped_plan *plan, void *hip_stream) {
    if (!plan || !plan->exec) return fail(PK_ERR_INVALID_ARG, "plan not captured");
    hipError_t err = hipGraphLaunch(plan->exec, (hipStream_t)hip_stream);
    if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(err));
    return PK_OK;
}

int pk_grouped_plan_info(const pk_grouped_plan *plan, int32_t *launches, int64_t *total_tiles, pk_params *chosen,
                         int32_t cap) {
    if (!plan) return fail(PK_ERR_INVALID_ARG, "null plan");
    const auto &lay = plan->layout;
    if (launches) *launches = (int32_t)lay.launches.size();
    if (total_tiles) {
        int64_t t = 0;
        for (const auto &L : lay.launches) t += L.total_tiles;
        *total_tiles = t;
    }
    if (chosen) {
        if (cap < (int32_t)lay.chosen.size()) return fail(PK_ERR_BUFFER_TOO_SMALL, "cap below the product count");
        std::copy(lay.chosen.begin(), lay.chosen.end(), chosen);
    }
    return PK_OK;
}

int pk_grouped_plan_kernel(const pk_grouped_plan *plan, int32_t i, const char **name) {
    if (!plan || !name) return fail(PK_ERR_INVALID_ARG, "null argument");
    if (i < 0 || i >= (int32_t)plan->layout.launches.size()) return fail(PK_ERR_INVALID_ARG, "launch index out of range");
    *name = plan->layout.launches[i].entry->name;
    return PK_OK;
}

void pk_grouped_plan_destroy(pk_grouped_plan *plan) { delete plan; }

int pk_matmul_batched(const pk_table *tbl, pk_dtype dtype, int32_t G, const int64_t *M, const int64_t *N,
                      const int64_t *K, const void *const *A, const int64_t *lda, const void *const *B,
                      const int64_t *ldb, void *const *C, const int64_t *ldc, const pk_params *per_group_or_null,
                      void *hip_stream) {
    pk_grouped_plan *plan = nullptr;
    int rc = pk_grouped_plan_create(tbl, dtype, G, M, N, K, A, lda, B, ldb, C, ldc, per_group_or_null,
                                    PK_POLICY_CASE, 0, &plan);
    if (rc != PK_OK) return rc;
    rc = pk_grouped_plan_run(plan, hip_stream);
    hipError_t err = hipStreamSynchronize((hipStream_t)hip_stream);
    pk_grouped_plan_destroy(plan);
    if (rc != PK_OK) return rc;
    if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(err));
    return PK_OK;
}

}  // extern "C"
