// Internal declarations of the pk library (host side).
//
// Symbolic part: integer polynomials, constraint systems, the quintuple and
// Algorithms 1 and 2 of Section 3.7, and the code-fragment families the
// algorithm is run on.  Runtime part: the registry of compiled kernel
// instances, the bound case table and the launch plumbing.
#pragma once

#include <cstdint>
#include <atomic>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "pk.h"
#include "kernels/kargs.hpp"

namespace pk {

// Largest M, N or K accepted: kernels index rows and columns in 32-bit
// integers, and a tile rounded up past the last row or column must still fit.
constexpr int64_t kMaxDim = 0x7fff0000;
// Largest number of shares of K a product is split into.
constexpr int kMaxSplits = 16;


// ------------------------------------------------------------------ errors
int fail(int code, const std::string &msg);  // stores msg for pk_last_error, returns code
void clear_error();

// ------------------------------------------------------------------ polynomials
// A monomial is a sorted list of (symbol id, exponent); the empty list is 1.
using Mono = std::vector<std::pair<int, int>>;

struct Poly {
    std::map<Mono, int64_t> t;  // monomial -> integer coefficient (no zero entries)

    static Poly constant(int64_t c);
    static Poly symbol(int id);
    Poly operator+(const Poly &o) const;
    Poly operator-(const Poly &o) const;
    Poly operator*(const Poly &o) const;
    Poly neg() const;
    bool is_const() const;
    int64_t const_value() const;
    // Value with every symbol given; vals[id] is the value of symbol id.
    int64_t eval(const std::vector<int64_t> &vals) const;
};

// Parses "2*s*B + 2", "(B0+1)^2", "-x"; symbol names are resolved through
// `lookup` (returns -1 for an unknown name).  Throws std::runtime_error.
Poly parse_poly(const std::string &text, const std::function<int(const std::string &)> &lookup);

// lhs <= rhs, or lhs < rhs when strict.
struct Constraint {
    Poly lhs, rhs;
    bool strict = false;
};
using System = std::vector<Constraint>;

// ------------------------------------------------------------------ families
enum SymKind { SYM_MACHINE = 0, SYM_PROGRAM = 1, SYM_DATA = 2, SYM_TABLE = 3 };

struct CounterDef {
    std::string name;
    bool performance = false;  // resource counter r_i otherwise
    int limit = -1;            // machine symbol R_i or P_i
    // value of the counter on the fragment after the strategies in `applied`
    std::function<Poly(uint32_t applied)> value;
};

struct StrategyDef {
    std::string name;
    bool on_ir = false;     // recorded in lambda when true
    uint32_t sigma = 0;     // bit c set: may improve counter c
};

// A code fragment S with its evaluation functions and strategies.
struct Family {
    std::vector<std::string> sym_names;
    std::vector<int> sym_kind;                  // SymKind per symbol
    std::vector<int64_t> lo, hi;                // interval domain of machine symbols
    std::vector<CounterDef> counters;           // gamma order: r_1..r_s, p_1..p_t
    std::vector<StrategyDef> strategies;        // omega order: O_1..O_w
    std::vector<int> point_syms;                // program/data symbols spanned by `points`
    std::vector<std::vector<int64_t>> points;   // finite domain of (program, data) values
    // value of a table symbol at a point (same order as point_syms); a
    // missing entry is reported as `missing_table_value`
    std::function<int64_t(int sym, const std::vector<int64_t> &point)> table;
    int64_t perf_one = 1;

    int sym(const std::string &name) const;     // id or -1
    std::string poly_str(const Poly &p) const;
    std::string constraint_str(const Constraint &c) const;
};

// Value reported for a table symbol with no compiled instance: large enough
// that no machine limit admits it.
constexpr int64_t missing_table_value = int64_t(1) << 40;

struct Leaf {
    uint32_t applied = 0;            // strategy bits (source and IR) = the variant
    std::vector<int> order;          // strategies in the order they were applied
    std::vector<int> lam;            // lambda: IR strategies applied
    System C;
};

struct SolveResult {
    std::vector<Leaf> leaves;  // output stack of Algorithm 1, head first
    int height = 0;            // height of the tree T(Q(S))
};

// Algorithms 1 and 2 on a family.  Consistency is decided exactly over the
// family's finite point set and the machine symbols' integer intervals.
SolveResult comprehensive_optimization(const Family &fam);
bool consistent(const Family &fam, const System &C);

// Evaluation of a system at a point of the family and fixed machine values.
// `machine_vals` is indexed by symbol id (non-machine entries ignored).
bool system_holds(const Family &fam, const System &C, const std::vector<int64_t> &point,
                  const std::vector<int64_t> &machine_vals);

std::string json_escape(const std::string &s);
std::string leaves_json(const Family &fam, const SolveResult &r);

// Parses the text description accepted by pk_co_solve.
Family parse_family(const std::string &spec);

// ------------------------------------------------------------------ registry
using MmArgs = pkk::MmArgs;
using KernelEntry = pkk::KernelEntry;

struct KernelResources {
    int vgpr = 0, agpr = 0, sgpr = 0, scratch = 0, lds = 0, occupancy = 0;
};

const std::vector<KernelEntry> &registry();
const KernelResources *resources_of(const char *name);
// registers one workgroup of `threads` work-items allocates on gfx950
// (unified VGPR file: arch VGPRs rounded to 4 plus AGPRs, granule 8, per lane)
int64_t regs_per_block(const KernelResources &r, int threads, int wave);

// ------------------------------------------------------------------ families of the matmul
// Builds the symbolic family for (family id, dtype); its table symbols read
// the registry and resources above.
Family matmul_family(int family, int dtype);
// E point of a pk_params for a family (order of Family::point_syms)
bool params_point(int family, const pk_params &p, std::vector<int64_t> *pt);
void point_params(int family, const std::vector<int64_t> &pt, pk_params *p);
// machine symbol values of a pk_machine, indexed like the family's symbols
std::vector<int64_t> machine_values(const Family &fam, const pk_machine &m);
// Does the variant's program fit at E (all its resource counters within the
// machine limits)?  This is code soundness without the case discussion.
bool variant_fits(const Family &fam, uint32_t variant, const std::vector<int64_t> &pt,
                  const std::vector<int64_t> &machine_vals);
const KernelEntry *find_instance(int family, int variant, int dtype, const std::vector<int64_t> &pt);
// The element-load twin of a single-launch MFMA instance (same program,
// rows read element by element), or null.
const KernelEntry *element_twin(const KernelEntry &e);
// The split-along-K form of a single-launch MFMA instance's wide program, or
// null (programs that are never split).
const KernelEntry *split_twin(const KernelEntry &e);

// Looks up, once per device and with that device current, the device address
// of the allocation-free entry point's workspace (noalloc.hip).
int noalloc_setup(int device);

// The several-steps 1D Jacobi instance of (dtype, bx, s), or null.
const KernelEntry *find_jacobi_fused(int dtype, int64_t bx, int64_t s);

// The one-launch polynomial-division instance named by a variant
// (PK_POLYDIV_FUSED, with or without PK_POLYDIV_WIDE) and (bx, s), or null.
const KernelEntry *find_polydiv_fused(int variant, int64_t bx, int64_t s);

}  // namespace pk

// The bound case table (opaque in the C ABI).
struct pk_table {
    std::shared_ptr<pk_costmodel> costmodel[3];  // for PK_POLICY_LEARNED, per pk_dtype, or null
    mutable std::atomic<int64_t> learned_selections{0}, learned_fallbacks{0}, learned_measured{0};
    // LEARNED: candidates predicted within this fraction of the best are
    // measured when the best two are that close (0 never measures)
    double learned_margin = 0.05;
    pk_machine machine;
    int device = -1;
    struct Part {
        int family = 0;
        int dtype = 0;
        bool supported = false;
        pk::Family fam;
        pk::SolveResult solved;
        std::vector<int64_t> mvals;                 // machine values by symbol id
        std::vector<int> first_leaf;                // per point: first satisfied leaf or -1
    };
    std::vector<Part> parts;  // PK_NUM_FAMILIES x 3 dtypes
    const Part *part(int family, int dtype) const;
    mutable std::mutex cache_mu;
    mutable std::map<std::tuple<int, int64_t, int64_t, int64_t, int>, pk_params> cache;
};
