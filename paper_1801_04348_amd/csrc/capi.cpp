// C ABI of the pk library: machine query, symbolic solve, case-table build
// and binding, lookup, and the matmul launch.  Nothing throws across the
// boundary: every entry point catches and returns a PK_ERR_* code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <stdexcept>

#include "pk_internal.hpp"
#include "select.hpp"

namespace pk {

namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}
void clear_error() { g_err.clear(); }

static int copy_out(const std::string &s, char *out, size_t cap, size_t *needed) {
    if (needed) *needed = s.size() + 1;
    if (!out || cap < s.size() + 1) return fail(PK_ERR_BUFFER_TOO_SMALL, "output buffer too small");
    std::memcpy(out, s.c_str(), s.size() + 1);
    return PK_OK;
}

// ------------------------------------------------------------------ instance lookup for a call
// Resolves params (or the case table) into a runnable instance.
int resolve(const pk_table *tbl, const pk_params *pin, int dtype, pk_params *pout, const KernelEntry **entry) {
    if (pin->family < 0 || pin->family >= PK_NUM_FAMILIES)
        return fail(PK_ERR_INVALID_ARG, "unknown family " + std::to_string(pin->family));
    const pk_table::Part *part = tbl->part(pin->family, dtype);
    if (!part || !part->supported)
        return fail(PK_ERR_UNSUPPORTED_DTYPE, "family " + std::to_string(pin->family) + " has no kernel for dtype " +
                                                  std::to_string(dtype));
    std::vector<int64_t> pt;
    if (!params_point(pin->family, *pin, &pt)) return fail(PK_ERR_INVALID_ARG, "parameters outside the family");
    auto it = std::find(part->fam.points.begin(), part->fam.points.end(), pt);
    if (it == part->fam.points.end())
        return fail(PK_ERR_INVALID_ARG, "program parameters outside the family's domain");
    const size_t idx = it - part->fam.points.begin();
    int leaf = pin->leaf;
    int variant = pin->variant;
    if (leaf >= 0) {
        if (leaf >= (int)part->solved.leaves.size()) return fail(PK_ERR_INVALID_ARG, "leaf index out of range");
        const Leaf &L = part->solved.leaves[leaf];
        if (!system_holds(part->fam, L.C, pt, part->mvals))
            return fail(PK_ERR_NO_FEASIBLE_BRANCH, "the leaf's system does not hold at these parameters");
        variant = (int)L.applied;
    } else if (variant >= 0) {
        if (!variant_fits(part->fam, (uint32_t)variant, pt, part->mvals))
            return fail(PK_ERR_NO_FEASIBLE_BRANCH, "the variant does not fit the machine at these parameters");
    } else {
        leaf = part->first_leaf[idx];
        if (leaf < 0) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no leaf of the case table holds at these parameters");
        variant = (int)part->solved.leaves[leaf].applied;
    }
    const KernelEntry *e = find_instance(pin->family, variant, dtype, pt);
    if (!e) return fail(PK_ERR_NOT_INSTANTIATED, "no compiled instance for these parameters");
    if (pin->ks < 0 || pin->ks > kMaxSplits || (pin->ks > 1 && !split_twin(*e)))
        return fail(PK_ERR_INVALID_ARG, "ks: shares of K are 0 or 1 (none), or up to " + std::to_string(kMaxSplits) +
                                            " for the MFMA programs that have a split form (up to " +
                                            std::to_string(pkk::kSplittableThreads) + " work-items)");
    *pout = *pin;
    point_params(pin->family, pt, pout);
    pout->ks = pin->ks > 1 ? pin->ks : 0;
    pout->leaf = leaf;
    pout->variant = variant;
    *entry = e;
    return PK_OK;
}

// Workgroups of an instance resident on one compute unit: wave slots
// (max_threads_cu / wave, a workgroup holding whole wavefronts), LDS and
// registers, and the runtime's workgroup limit -- unless that limit is no
// more than max_threads_cu / max_threads_block, a figure that only describes
// full-size workgroups (one HIP runtime reports 2 for gfx950, another 32).
int64_t blocks_per_cu(const pk_machine &m, const KernelEntry &e) {
    const KernelResources *r = resources_of(e.name);
    const int64_t wave = m.wave > 0 ? m.wave : 64;
    const int64_t waves = (e.threads + wave - 1) / wave;
    int64_t b = m.max_threads_cu > 0 ? std::max<int64_t>(1, m.max_threads_cu / wave) / waves : 32;
    const bool derived = m.max_threads_block > 0 && m.max_threads_cu > 0 &&
                         (int64_t)m.max_blocks_cu * m.max_threads_block <= m.max_threads_cu;
    if (m.max_blocks_cu > 0 && !derived) b = std::min<int64_t>(b, m.max_blocks_cu);
    if (e.lds_bytes > 0) b = std::min<int64_t>(b, m.lds_cu / e.lds_bytes);
    if (r) {
        int64_t rb = regs_per_block(*r, e.threads, m.wave > 0 ? m.wave : 64);
        if (rb > 0) b = std::min<int64_t>(b, m.regs_cu / rb);
    }
    return std::max<int64_t>(b, 1);
}

// One workgroup per tile for the MFMA programs, matrix addition, 1D Jacobi
// and transposition (their tile loops then run once): for the HBM-bound
// programs the hardware keeps the compute units full with fresh workgroups,
// which keeps more loads in flight than a resident grid striding over the
// tiles (matrix addition of order 2^14: 6.3 against 5.4 TB/s; transposition
// of order 2^14, best program: 4.9 against 4.7 TB/s; Jacobi a few per cent).
// The other programs stride over the tiles with a resident grid.
static bool one_tile_per_workgroup(const KernelEntry &e) {
    return e.family == PK_FAMILY_MFMA || e.family == PK_FAMILY_MADD || e.family == PK_FAMILY_JACOBI ||
           e.family == PK_FAMILY_TRANSPOSE;
}

int64_t grid_of(const pk_machine &m, const KernelEntry &e, int64_t M, int64_t N) {
    const int64_t tiles = ((M + e.tile_m - 1) / e.tile_m) * ((N + e.tile_n - 1) / e.tile_n);
    if (one_tile_per_workgroup(e)) return tiles;
    // VALU: a workgroup-stride loop over tiles, grid = resident capacity
    return std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)m.cu_count * blocks_per_cu(m, e)));
}

// Resident workgroups of a kernel per compute unit for a launch on the
// current device: the HIP runtime's occupancy calculator, which reads the
// kernel's actual register, LDS and wave needs against the hardware (some
// runtimes report a block register budget of half the register file, which
// the case table's model uses as reported); cached per kernel.  Falls back
// to the model's count if the query fails.
int64_t live_blocks_per_cu(const pk_machine &m, const KernelEntry &e) {
    static std::mutex mu;
    static std::map<const void *, int64_t> cache;
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find(e.fn);
        if (it != cache.end()) return it->second;
    }
    int n = 0;
    int64_t b = blocks_per_cu(m, e);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, e.fn, e.threads, 0) == hipSuccess && n > 0) b = n;
    else (void)hipGetLastError();
    std::lock_guard<std::mutex> lock(mu);
    cache[e.fn] = b;
    return b;
}

int64_t launch_grid(const pk_machine &m, const KernelEntry &e, int64_t M, int64_t N) {
    const int64_t tiles = ((M + e.tile_m - 1) / e.tile_m) * ((N + e.tile_n - 1) / e.tile_n);
    if (one_tile_per_workgroup(e)) return tiles;
    return std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)m.cu_count * live_blocks_per_cu(m, e)));
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Rows aligned for the MFMA programs' wide loads: 16-byte loads along the
// rows of A and B (leading dimensions multiples of 4 f32 / 8 bf16 elements,
// 16-byte aligned bases).  Otherwise the programs read element by element
// (same arithmetic, same summation order).
bool wide_rows(int dtype, const void *A, int64_t lda, const void *B, int64_t ldb) {
    const int64_t vec = dtype == PK_BF16 ? 8 : 4;
    return aligned16(A) && lda % vec == 0 && aligned16(B) && ldb % vec == 0;
}

int launch(const pk_machine &m, const KernelEntry &e0, const MmArgs &args, hipStream_t stream) {
    const KernelEntry *pe = &e0;
    MmArgs a = args;
    if (e0.family != PK_FAMILY_MFMA || a.K <= 0 || a.splits < 2) a.splits = 0;
    if (e0.family == PK_FAMILY_MFMA && !args.vec) {  // rows not aligned: the element-load twin (it splits in place)
        pe = element_twin(e0);
        if (!pe) return fail(PK_ERR_NOT_INSTANTIATED, std::string("no element-load twin of ") + e0.name);
    } else if (a.splits > 1) {  // shares of K: the wide program's split form
        pe = split_twin(e0);
        if (!pe) return fail(PK_ERR_INVALID_ARG, std::string("no split form of ") + e0.name);
    }
    const KernelEntry &e = *pe;
    const int64_t grid = launch_grid(m, e, args.M, args.N) * std::max(a.splits, 1);
    if (grid <= 0) return PK_OK;
    if (grid > 0x7fffffff) return fail(PK_ERR_INVALID_ARG, "grid too large");
    if (a.splits > 1 && !a.accumulate) {  // the shares add into C: clear it first
        int rc = zero_matrix(m, a.C, a.ldc, a.M, a.N, stream);
        if (rc != PK_OK) return rc;
    }
    void *kargs[] = {&a};
    hipError_t err = hipLaunchKernel(e.fn, dim3((unsigned)grid), dim3((unsigned)e.threads), kargs, 0, stream);
    if (err != hipSuccess)
        return fail(PK_ERR_HIP, std::string("hipLaunchKernel(") + e.name + "): " + hipGetErrorString(err));
    return PK_OK;
}

}  // namespace pk

using namespace pk;

// ------------------------------------------------------------------ table
const pk_table::Part *pk_table::part(int family, int dtype) const {
    for (const auto &p : parts)
        if (p.family == family && p.dtype == dtype) return &p;
    return nullptr;
}

extern "C" {

const char *pk_last_error(void) { return g_err.c_str(); }

const char *pk_version(void) { return "pk 0.1 (gfx950)"; }

int pk_instance_count(void) { return (int)registry().size(); }

const char *pk_instance_name(int i) {
    if (i < 0 || i >= (int)registry().size()) return nullptr;
    return registry()[i].name;
}

int pk_machine_query(int device, pk_machine *out) {
    if (!out) return fail(PK_ERR_INVALID_ARG, "null output");
    hipDeviceProp_t p;
    hipError_t err = hipGetDeviceProperties(&p, device);
    if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("hipGetDeviceProperties: ") + hipGetErrorString(err));
    std::memset(out, 0, sizeof *out);
    out->wave = p.warpSize;
    out->lds_block = (int64_t)p.sharedMemPerBlock;
    out->lds_cu = (int64_t)p.maxSharedMemoryPerMultiProcessor;
    out->regs_block = p.regsPerBlock;
    out->regs_cu = p.regsPerMultiprocessor;
    out->max_threads_block = p.maxThreadsPerBlock;
    out->max_threads_cu = p.maxThreadsPerMultiProcessor;
    out->max_blocks_cu = p.maxBlocksPerMultiProcessor;
    out->cu_count = p.multiProcessorCount;
    out->clock_khz = p.clockRate;
    std::strncpy(out->arch, p.gcnArchName, sizeof out->arch - 1);
    return PK_OK;
}

int pk_co_solve(const char *spec, char *out, size_t cap, size_t *needed) {
    if (!spec) return fail(PK_ERR_INVALID_ARG, "null spec");
    try {
        Family fam = parse_family(spec);
        SolveResult r = comprehensive_optimization(fam);
        return copy_out(leaves_json(fam, r), out, cap, needed);
    } catch (const std::exception &ex) {
        return fail(PK_ERR_PARSE, ex.what());
    }
}

int pk_case_table_build(int device, const pk_machine *override_or_null, pk_table **out) {
    if (!out) return fail(PK_ERR_INVALID_ARG, "null output");
    *out = nullptr;
    pk_machine m;
    if (override_or_null) {
        m = *override_or_null;
    } else {
        int rc = pk_machine_query(device, &m);
        if (rc != PK_OK) return rc;
        // the library's set-up on this device: the workspace address of the
        // allocation-free entry point
        rc = noalloc_setup(device);
        if (rc != PK_OK) return rc;
    }
    if (m.wave <= 0 || m.cu_count <= 0 || m.max_threads_block <= 0)
        return fail(PK_ERR_INVALID_ARG, "machine descriptor has non-positive wave, CU count or thread limit");
    try {
        std::unique_ptr<pk_table> t(new pk_table);
        t->machine = m;
        t->device = device;
        for (int family = 0; family < PK_NUM_FAMILIES; ++family)
            for (int dtype : {PK_F32, PK_I32, PK_BF16}) {
                pk_table::Part part;
                part.family = family;
                part.dtype = dtype;
                const bool ok = family == PK_FAMILY_MFMA      ? true
                                : family == PK_FAMILY_POLYDIV ? dtype == PK_I32
                                                              : (dtype == PK_F32 || dtype == PK_I32);
                part.supported = ok;
                if (ok) {
                    part.fam = matmul_family(family, dtype);
                    part.solved = comprehensive_optimization(part.fam);
                    part.mvals = machine_values(part.fam, m);
                    part.first_leaf.assign(part.fam.points.size(), -1);
                    for (size_t i = 0; i < part.fam.points.size(); ++i)
                        for (size_t l = 0; l < part.solved.leaves.size(); ++l)
                            if (system_holds(part.fam, part.solved.leaves[l].C, part.fam.points[i], part.mvals)) {
                                part.first_leaf[i] = (int)l;
                                break;
                            }
                }
                t->parts.push_back(std::move(part));
            }
        *out = t.release();
        return PK_OK;
    } catch (const std::exception &ex) {
        return fail(PK_ERR_INVALID_ARG, std::string("case table: ") + ex.what());
    }
}

void pk_case_table_free(pk_table *tbl) { delete tbl; }

int pk_case_table_describe(const pk_table *tbl, char *out, size_t cap, size_t *needed) {
    if (!tbl) return fail(PK_ERR_INVALID_ARG, "null table");
    const pk_machine &m = tbl->machine;
    std::ostringstream o;
    o << "{\"machine\":{\"wave\":" << m.wave << ",\"lds_block\":" << m.lds_block << ",\"lds_cu\":" << m.lds_cu
      << ",\"regs_block\":" << m.regs_block << ",\"regs_cu\":" << m.regs_cu
      << ",\"max_threads_block\":" << m.max_threads_block << ",\"max_threads_cu\":" << m.max_threads_cu
      << ",\"max_blocks_cu\":" << m.max_blocks_cu << ",\"cu_count\":" << m.cu_count << ",\"clock_khz\":" << m.clock_khz
      << ",\"arch\":\"" << json_escape(m.arch) << "\"},\"parts\":[";
    bool first = true;
    for (const auto &p : tbl->parts) {
        if (!p.supported) continue;
        if (!first) o << ",";
        first = false;
        o << "{\"family\":" << p.family << ",\"dtype\":" << p.dtype << ",\"symbols\":[";
        for (size_t s = 0; s < p.fam.sym_names.size(); ++s)
            o << (s ? "," : "") << "[\"" << p.fam.sym_names[s] << "\"," << p.fam.sym_kind[s] << "]";
        o << "],\"counters\":[";
        for (size_t c = 0; c < p.fam.counters.size(); ++c)
            o << (c ? "," : "") << "\"" << p.fam.counters[c].name << "\"";
        o << "],\"strategies\":[";
        for (size_t c = 0; c < p.fam.strategies.size(); ++c)
            o << (c ? "," : "") << "\"" << p.fam.strategies[c].name << "\"";
        o << "],\"points\":[";
        for (size_t i = 0; i < p.fam.points.size(); ++i) {
            o << (i ? "," : "") << "[";
            for (size_t k = 0; k < p.fam.points[i].size(); ++k) o << (k ? "," : "") << p.fam.points[i][k];
            o << "]";
        }
        o << "],\"tables\":{";
        bool ft = true;
        for (size_t s = 0; s < p.fam.sym_names.size(); ++s) {
            if (p.fam.sym_kind[s] != SYM_TABLE) continue;
            o << (ft ? "" : ",") << "\"" << p.fam.sym_names[s] << "\":[";
            ft = false;
            for (size_t i = 0; i < p.fam.points.size(); ++i) o << (i ? "," : "") << p.fam.table((int)s, p.fam.points[i]);
            o << "]";
        }
        o << "},\"first_leaf\":[";
        for (size_t i = 0; i < p.first_leaf.size(); ++i) o << (i ? "," : "") << p.first_leaf[i];
        o << "],\"solution\":" << leaves_json(p.fam, p.solved) << "}";
    }
    o << "],\"instances\":[";
    const auto &reg = registry();
    for (size_t i = 0; i < reg.size(); ++i) {
        const KernelEntry &e = reg[i];
        const KernelResources *r = resources_of(e.name);
        o << (i ? "," : "") << "{\"name\":\"" << e.name << "\",\"family\":" << e.family << ",\"variant\":" << e.variant
          << ",\"dtype\":" << e.dtype << ",\"bx\":" << e.bx << ",\"by\":" << e.by << ",\"s\":" << e.s
          << ",\"sy\":" << e.sy
          << ",\"bk\":" << e.bk << ",\"bm\":" << e.bm << ",\"bn\":" << e.bn << ",\"wm\":" << e.wm << ",\"wn\":" << e.wn
          << ",\"threads\":" << e.threads << ",\"lds_bytes\":" << e.lds_bytes << ",\"tile_m\":" << e.tile_m
          << ",\"tile_n\":" << e.tile_n;
        if (r)
            o << ",\"vgpr\":" << r->vgpr << ",\"agpr\":" << r->agpr << ",\"sgpr\":" << r->sgpr
              << ",\"scratch\":" << r->scratch << ",\"lds_compiled\":" << r->lds << ",\"occupancy\":" << r->occupancy;
        o << "}";
    }
    o << "]}";
    return copy_out(o.str(), out, cap, needed);
}

int pk_case_table_lookup(const pk_table *tbl, pk_dtype dtype, const pk_params *p, int32_t *leaf_out,
                         int32_t *variant_out) {
    if (!tbl || !p) return fail(PK_ERR_INVALID_ARG, "null argument");
    if (p->family < 0 || p->family >= PK_NUM_FAMILIES) return fail(PK_ERR_INVALID_ARG, "unknown family");
    const pk_table::Part *part = tbl->part(p->family, dtype);
    if (!part || !part->supported) return fail(PK_ERR_UNSUPPORTED_DTYPE, "family has no kernel for this dtype");
    std::vector<int64_t> pt;
    if (!params_point(p->family, *p, &pt)) return fail(PK_ERR_INVALID_ARG, "parameters outside the family");
    auto it = std::find(part->fam.points.begin(), part->fam.points.end(), pt);
    if (it == part->fam.points.end()) return fail(PK_ERR_INVALID_ARG, "program parameters outside the domain");
    const int leaf = part->first_leaf[it - part->fam.points.begin()];
    if (leaf < 0) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no leaf holds at these parameters");
    if (leaf_out) *leaf_out = leaf;
    if (variant_out) *variant_out = (int32_t)part->solved.leaves[leaf].applied;
    return PK_OK;
}

int pk_select(const pk_table *tbl, pk_dtype dtype, int64_t M, int64_t N, int64_t K, int policy, pk_params *out) {
    if (!tbl || !out) return fail(PK_ERR_INVALID_ARG, "null argument");
    if (M < 0 || N < 0 || K < 0) return fail(PK_ERR_INVALID_ARG, "negative dimension");
    try {
        return select_params(tbl, (int)dtype, M, N, K, policy, true, out);
    } catch (const std::exception &ex) {
        return fail(PK_ERR_INVALID_ARG, ex.what());
    }
}

int pk_select_operands(const pk_table *tbl, pk_dtype dtype, const void *A, int64_t lda, const void *B, int64_t ldb,
                       int64_t M, int64_t N, int64_t K, int policy, pk_params *out) {
    if (!tbl || !out) return fail(PK_ERR_INVALID_ARG, "null argument");
    if (M <= 0 || N <= 0 || K < 0) return fail(PK_ERR_INVALID_ARG, "M and N must be positive, K non-negative");
    if (K > 0 && (!A || !B || lda < K || ldb < N)) return fail(PK_ERR_INVALID_ARG, "null A/B or lda < K or ldb < N");
    try {
        return select_params(tbl, (int)dtype, M, N, K, policy, false, out, K > 0 ? A : nullptr, lda, B, ldb);
    } catch (const std::exception &ex) {
        return fail(PK_ERR_INVALID_ARG, ex.what());
    }
}

int pk_measure(const pk_table *tbl, pk_dtype dtype, const void *A, int64_t lda, const void *B, int64_t ldb, void *C,
               int64_t ldc, int64_t M, int64_t N, int64_t K, pk_params *params_out, double *seconds_out, int cap,
               int *n) {
    if (!tbl || !n) return fail(PK_ERR_INVALID_ARG, "null argument");
    if (M <= 0 || N <= 0 || K < 0) return fail(PK_ERR_INVALID_ARG, "M and N must be positive, K non-negative");
    if (A && (!B || !C || lda < K || ldb < N || ldc < N)) return fail(PK_ERR_INVALID_ARG, "operands inconsistent");
    try {
        std::vector<Candidate> cands = feasible(tbl, (int)dtype, M, N, K, A, lda, B, ldb);
        *n = (int)cands.size();
        if (cands.empty()) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no leaf of the case table holds");
        if (cap < (int)cands.size()) return fail(PK_ERR_BUFFER_TOO_SMALL, "cap below the number of candidates");
        std::vector<double> secs;
        Operands ops{A, lda, B, ldb, C, ldc};
        int best = -1;
        const int rc = time_candidates(tbl, (int)dtype, M, N, K, cands, &secs, A ? &ops : nullptr, &best);
        if (rc != PK_OK) return rc;
        for (size_t i = 0; i < cands.size(); ++i) {
            if (params_out) fill_params(tbl, cands[i], (int)dtype, &params_out[i]);
            if (seconds_out) seconds_out[i] = secs[i];
        }
        return PK_OK;
    } catch (const std::exception &ex) {
        return fail(PK_ERR_HIP, ex.what());
    }
}

const char *pk_kernel_name(const pk_table *tbl, const pk_params *p, pk_dtype dtype) {
    if (!tbl || !p) {
        fail(PK_ERR_INVALID_ARG, "null argument");
        return nullptr;
    }
    pk_params q;
    const KernelEntry *e = nullptr;
    if (p->family == PK_FAMILY_POLYDIV && p->variant >= 0 && (p->variant & PK_POLYDIV_FUSED)) {
        e = find_polydiv_fused(p->variant, p->bx, p->s);
        if (!e) fail(PK_ERR_NOT_INSTANTIATED, "no one-launch division instance for these parameters");
        return e ? e->name : nullptr;
    }
    if (p->family == PK_FAMILY_JACOBI && p->variant >= 0 && (p->variant & PK_JACOBI_FUSED)) {
        e = find_jacobi_fused((int)dtype, p->bx, p->s);
        if (!e) fail(PK_ERR_NOT_INSTANTIATED, "no several-steps Jacobi instance for these parameters");
        return e ? e->name : nullptr;
    }
    if (resolve(tbl, p, (int)dtype, &q, &e) != PK_OK) return nullptr;
    return e->name;
}

int pk_estimate(const pk_table *tbl, const pk_params *p, pk_dtype dtype, int64_t M, int64_t N, int64_t K, int wide,
                double *seconds) {
    if (!tbl || !p || !seconds) return fail(PK_ERR_INVALID_ARG, "null argument");
    if (M < 0 || N < 0 || K < 0) return fail(PK_ERR_INVALID_ARG, "negative dimension");
    if (p->family != PK_FAMILY_VALU && p->family != PK_FAMILY_VALU2 && p->family != PK_FAMILY_MFMA)
        return fail(PK_ERR_INVALID_ARG, "estimates cover the matmul families");
    pk_params q;
    const KernelEntry *e = nullptr;
    int rc = resolve(tbl, p, (int)dtype, &q, &e);
    if (rc != PK_OK) return rc;
    *seconds = estimate_seconds(tbl->machine, *e, (int)dtype, M, N, K, wide != 0, std::max(q.ks, 1));
    return PK_OK;
}

int pk_launch_shape(const pk_table *tbl, const pk_params *p, pk_dtype dtype, int64_t M, int64_t N, int64_t K,
                    int64_t *grid, int32_t *block, int64_t *lds_bytes) {
    (void)K;
    if (!tbl || !p) return fail(PK_ERR_INVALID_ARG, "null argument");
    pk_params q;
    const KernelEntry *e = nullptr;
    if (p->family == PK_FAMILY_POLYDIV && p->variant >= 0 && (p->variant & PK_POLYDIV_FUSED)) {
        e = find_polydiv_fused(p->variant, p->bx, p->s);
        if (!e) return fail(PK_ERR_NOT_INSTANTIATED, "no one-launch division instance for these parameters");
    } else {
        int rc = resolve(tbl, p, (int)dtype, &q, &e);
        if (rc != PK_OK) return rc;
    }
    if (grid) *grid = grid_of(tbl->machine, *e, M, N) * (e->family == PK_FAMILY_MFMA ? std::max(q.ks, 1) : 1);
    if (block) *block = e->threads;
    if (lds_bytes) *lds_bytes = e->lds_bytes;
    return PK_OK;
}

int pk_matmul(const pk_table *tbl, const pk_params *params_or_null, pk_dtype dtype, const void *A, int64_t lda,
              const void *B, int64_t ldb, void *C, int64_t ldc, int64_t M, int64_t N, int64_t K, int accumulate,
              void *hip_stream) {
    if (!tbl) return fail(PK_ERR_INVALID_ARG, "null table");
    if (M < 0 || N < 0 || K < 0) return fail(PK_ERR_INVALID_ARG, "negative dimension");
    if (M > kMaxDim || N > kMaxDim || K > kMaxDim) return fail(PK_ERR_INVALID_ARG, "dimension above 2^31 - 2^16");
    if (dtype != PK_F32 && dtype != PK_I32 && dtype != PK_BF16) return fail(PK_ERR_UNSUPPORTED_DTYPE, "unknown dtype");
    if (M == 0 || N == 0) return PK_OK;
    if (!C || ldc < N) return fail(PK_ERR_INVALID_ARG, "null C or ldc < N");
    if (K > 0 && (!A || !B || lda < K || ldb < N)) return fail(PK_ERR_INVALID_ARG, "null A/B or lda < K or ldb < N");
    try {
        pk_params sel;
        if (!params_or_null) {
            int rc = select_params(tbl, (int)dtype, M, N, K, PK_POLICY_CASE, false, &sel, A, lda, B, ldb);
            if (rc != PK_OK) return rc;
            params_or_null = &sel;
        }
        if (params_or_null->family != PK_FAMILY_VALU && params_or_null->family != PK_FAMILY_VALU2 &&
            params_or_null->family != PK_FAMILY_MFMA)
            return fail(PK_ERR_INVALID_ARG, "parameters of a family that is not a product");
        pk_params q;
        const KernelEntry *e = nullptr;
        int rc = resolve(tbl, params_or_null, (int)dtype, &q, &e);
        if (rc != PK_OK) return rc;
        const bool wide = wide_rows((int)dtype, A, lda, B, ldb);
        if (e->family == PK_FAMILY_MFMA && !wide && !element_twin(*e)) {
            // a program with no element-load form (it would spill) on rows
            // not aligned for its wide loads: the CASE choice for these
            // operands runs instead (pk_select, which sees no operands, may
            // return such a program)
            rc = select_params(tbl, (int)dtype, M, N, K, PK_POLICY_CASE, false, &sel, A, lda, B, ldb);
            if (rc != PK_OK) return rc;
            rc = resolve(tbl, &sel, (int)dtype, &q, &e);
            if (rc != PK_OK) return rc;
        }
        MmArgs args{A, B, C, lda, ldb, ldc, (int32_t)M, (int32_t)N, (int32_t)K, accumulate ? 1 : 0, wide ? 1 : 0,
                    q.ks, 0};
        return launch(tbl->machine, *e, args, (hipStream_t)hip_stream);
    } catch (const std::exception &ex) {
        return fail(PK_ERR_INVALID_ARG, ex.what());
    }
}

}  // extern "C"
