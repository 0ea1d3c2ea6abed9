// Many independent products in one persistent launch per tile configuration.
//
// A plan fixes, once, everything a grouped launch needs: for every product its
// leaf and program parameters (given per product, or else one program for
// all of them: among the MFMA points with grouped instances that fit every
// product, the one whose tiles cost the least compute-unit time in total, or
// under EXHAUSTIVE the one whose plan runs fastest when timed),
// its descriptor
// (pointers, leading dimensions, sizes, whether rows are aligned for the wide
// loads, first global tile index), and a tile -> product map.  Products are
// partitioned by tile configuration; each part is one persistent launch whose
// workgroups stride over that part's tiles.  Descriptors and maps are staged in
// pinned host memory and copied to the device when the plan is created, so
// running a plan allocates nothing and does not synchronise: it can be
// captured in a HIP graph, and pk_grouped_plan_capture does that itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <stdexcept>

#include "pk_internal.hpp"
#include "select.hpp"

using pkk::GroupArgs;
using pkk::GroupDesc;

struct pk_grouped_plan {
    int dtype = 0;
    int device = -1;
    int accumulate = 0;
    struct Launch {
        const pk::KernelEntry *entry = nullptr;
        int64_t first_desc = 0, ndesc = 0;     // range in the descriptor array
        int64_t first_tile = 0, total_tiles = 0;  // range in the tile map
        int64_t grid = 0;
    };
    std::vector<Launch> launches;
    std::vector<pk_params> chosen;  // per product, in the caller's order
    void *host = nullptr;           // pinned staging copy
    void *dev = nullptr;            // descriptors, then tile maps
    size_t bytes = 0;
    int64_t ndesc = 0;
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

// MFMA points with grouped instances, for the dtype
static bool grouped_instance(int dtype, int variant, const std::vector<int64_t> &pt, const KernelEntry **e) {
    *e = find_instance(PK_FAMILY_MFMA, variant | PK_MFMA_GROUPED, dtype, pt);
    return *e != nullptr;
}

static bool aligned_rows(int dtype, const void *A, int64_t lda, const void *B, int64_t ldb) {
    return wide_rows(dtype, A, lda, B, ldb);
}

}  // namespace pk

using namespace pk;

extern "C" int pk_grouped_plan_run(const pk_grouped_plan *plan, void *hip_stream);

namespace pk {
// seconds per run of a plan: one untimed run, then the median of three
static int time_plan(const pk_grouped_plan *plan, double *secs) {
    hipError_t err = hipSetDevice(plan->device);
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (err == hipSuccess) err = hipStreamCreate(&s);
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    int rc = err == hipSuccess ? pk_grouped_plan_run(plan, s) : PK_ERR_HIP;
    float t[3] = {0.f, 0.f, 0.f};
    for (int i = 0; i < 3 && rc == PK_OK && err == hipSuccess; ++i) {
        err = hipEventRecord(e0, s);
        if (err == hipSuccess) rc = pk_grouped_plan_run(plan, s);
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
}  // namespace pk

extern "C" {

int pk_grouped_plan_create(const pk_table *tbl, pk_dtype dtype, int32_t G, const int64_t *M, const int64_t *N,
                           const int64_t *K, const void *const *A, const int64_t *lda, const void *const *B,
                           const int64_t *ldb, void *const *C, const int64_t *ldc,
                           const pk_params *per_group_or_null, int policy, int accumulate,
                           pk_grouped_plan **out) {
    if (!tbl || !out || G < 0 || (G > 0 && (!M || !N || !K || !A || !lda || !B || !ldb || !C || !ldc)))
        return fail(PK_ERR_INVALID_ARG, "null argument or negative group count");
    if (dtype != PK_F32 && dtype != PK_BF16) return fail(PK_ERR_UNSUPPORTED_DTYPE, "grouped products: f32 or bf16");
    if (tbl->device < 0) return fail(PK_ERR_INVALID_ARG, "grouped plans need a table bound to a device");
    if (policy != PK_POLICY_CASE && policy != PK_POLICY_LEARNED && policy != PK_POLICY_EXHAUSTIVE)
        return fail(PK_ERR_INVALID_ARG, "grouped plans: policy CASE, LEARNED or EXHAUSTIVE");
    if (policy == PK_POLICY_EXHAUSTIVE && accumulate && !per_group_or_null)
        return fail(PK_ERR_INVALID_ARG, "grouped plans: EXHAUSTIVE selection writes C, so not with accumulate");
    *out = nullptr;
    try {
        std::unique_ptr<pk_grouped_plan> plan(new pk_grouped_plan);
        plan->dtype = (int)dtype;
        plan->device = tbl->device;
        plan->accumulate = accumulate ? 1 : 0;
        const pk_table::Part *part = tbl->part(PK_FAMILY_MFMA, (int)dtype);
        // choose per product: candidates are the feasible MFMA (leaf, E) pairs
        // with grouped instances; the policy ranks them (one batched
        // prediction for all products under LEARNED)
        std::map<const KernelEntry *, std::vector<int>> by_entry;
        plan->chosen.assign(G, pk_params{});
        std::vector<std::vector<Candidate>> okc(G);
        std::vector<std::vector<const KernelEntry *>> okg(G);  // the grouped instance of each
        for (int g = 0; g < G; ++g) {
            if (M[g] < 0 || N[g] < 0 || K[g] < 0 || M[g] > kMaxDim || N[g] > kMaxDim || K[g] > kMaxDim)
                return fail(PK_ERR_INVALID_ARG, "bad size in product " + std::to_string(g));
            if (M[g] == 0 || N[g] == 0) continue;
            if (!C[g] || ldc[g] < N[g] || (K[g] > 0 && (!A[g] || !B[g] || lda[g] < K[g] || ldb[g] < N[g])))
                return fail(PK_ERR_INVALID_ARG, "bad operands in product " + std::to_string(g));
            if (per_group_or_null) continue;
            const KernelEntry *ge = nullptr;
            for (const auto &c : feasible(tbl, (int)dtype, M[g], N[g], K[g]))
                if (c.family == PK_FAMILY_MFMA &&
                    grouped_instance((int)dtype, c.variant, part->fam.points[c.point], &ge)) {
                    okc[g].push_back(c);
                    okg[g].push_back(ge);
                }
            if (okc[g].empty())
                return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no grouped program fits product " + std::to_string(g));
        }
        // one program for the whole plan: the one whose tiles cost the least
        // compute-unit time summed over the products (a persistent launch runs
        // products side by side, so per-product launch latency does not
        // count; one launch instead of one per program chosen)
        const KernelEntry *plan_entry = nullptr;
        if (!per_group_or_null) {
            std::map<const KernelEntry *, std::pair<double, int>> total;  // work, products it fits
            int live = 0;
            for (int g = 0; g < G; ++g) {
                if (M[g] == 0 || N[g] == 0) continue;
                ++live;
                for (size_t i = 0; i < okc[g].size(); ++i) {
                    // the cost of the grouped instance, which is what runs
                    auto &t = total[okc[g][i].entry];
                    t.first += tile_work_seconds(tbl->machine, *okg[g][i], (int)dtype, M[g], N[g], K[g]);
                    t.second += 1;
                }
            }
            double best = 0.0;
            for (const auto &kv : total)
                if (kv.second.second == live && (!plan_entry || kv.second.first < best)) {
                    plan_entry = kv.first;
                    best = kv.second.first;
                }
            if (policy == PK_POLICY_EXHAUSTIVE && live > 0) {
                // the auto-tuner over the programs that could run every
                // product: each point whose case-table leaf holds for all of
                // them, with each LDS-stage variant whose resources fit (as a
                // forced variant would run); a plan of each is timed on the
                // plan's own operands and the fastest kept
                bool have = false;
                pk_params best_p{};
                double best_s = 0.0;
                for (const auto &kv : total) {
                    if (kv.second.second != live) continue;
                    const KernelEntry *e = kv.first;
                    for (int v : {0, (int)PK_MFMA_SINGLE}) {
                        pk_params proto{};
                        proto.family = PK_FAMILY_MFMA;
                        proto.leaf = -1;
                        proto.variant = v;
                        proto.bm = e->bm;
                        proto.bn = e->bn;
                        proto.bk = e->bk;
                        proto.wm = e->wm;
                        proto.wn = e->wn;
                        const std::vector<pk_params> ps(G, proto);
                        pk_grouped_plan *trial = nullptr;
                        int rc = pk_grouped_plan_create(tbl, dtype, G, M, N, K, A, lda, B, ldb, C, ldc, ps.data(),
                                                        PK_POLICY_CASE, 0, &trial);
                        if (rc == PK_ERR_NO_FEASIBLE_BRANCH || rc == PK_ERR_NOT_INSTANTIATED) continue;
                        if (rc != PK_OK) return rc;
                        std::unique_ptr<pk_grouped_plan> owned(trial);
                        double secs = 0.0;
                        rc = time_plan(trial, &secs);
                        if (rc != PK_OK) return rc;
                        if (!have || secs < best_s) {
                            have = true;
                            best_s = secs;
                            best_p = proto;
                        }
                    }
                }
                if (!have) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no grouped program fits every product");
                const std::vector<pk_params> ps(G, best_p);
                return pk_grouped_plan_create(tbl, dtype, G, M, N, K, A, lda, B, ldb, C, ldc, ps.data(), PK_POLICY_CASE,
                                              0, out);
            }
        }
        for (int g = 0; g < G; ++g) {
            if (M[g] == 0 || N[g] == 0) continue;
            pk_params p;
            if (per_group_or_null) {
                p = per_group_or_null[g];
                if (p.family != PK_FAMILY_MFMA)
                    return fail(PK_ERR_UNSUPPORTED_DTYPE, "grouped launches run MFMA programs only");
                pk_params q;
                const KernelEntry *e0 = nullptr;
                int rc = resolve(tbl, &p, (int)dtype, &q, &e0);
                if (rc != PK_OK) return rc;
                p = q;
            } else {
                const auto &ok = okc[g];
                int pick = -1;
                for (size_t i = 0; i < ok.size(); ++i)
                    if (ok[i].entry == plan_entry) pick = (int)i;
                if (pick < 0) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no grouped program fits every product");
                fill_params(tbl, ok[pick], (int)dtype, &p);
            }
            std::vector<int64_t> pt;
            params_point(PK_FAMILY_MFMA, p, &pt);
            const KernelEntry *e = nullptr;
            if (!grouped_instance((int)dtype, p.variant, pt, &e))
                return fail(PK_ERR_NOT_INSTANTIATED, "no grouped instance for product " + std::to_string(g));
            plan->chosen[g] = p;
            by_entry[e].push_back(g);
        }
        // descriptors and tile maps, one contiguous block per launch
        std::vector<GroupDesc> descs;
        std::vector<int32_t> tmap;
        for (auto &kv : by_entry) {
            const KernelEntry *e = kv.first;
            pk_grouped_plan::Launch L;
            L.entry = e;
            L.first_desc = (int64_t)descs.size();
            L.first_tile = (int64_t)tmap.size();
            int64_t tiles = 0;
            for (int g : kv.second) {
                GroupDesc d;
                std::memset(&d, 0, sizeof d);
                d.A = A[g];
                d.B = B[g];
                d.C = C[g];
                d.lda = lda[g];
                d.ldb = ldb[g];
                d.ldc = ldc[g];
                d.M = (int32_t)M[g];
                d.N = (int32_t)N[g];
                d.K = (int32_t)K[g];
                d.vec = aligned_rows((int)dtype, A[g], lda[g], B[g], ldb[g]) ? 1 : 0;
                d.tile_start = tiles;
                d.tiles_n = (int32_t)((N[g] + e->tile_n - 1) / e->tile_n);
                const int64_t t = ((M[g] + e->tile_m - 1) / e->tile_m) * d.tiles_n;
                const int32_t local = (int32_t)(descs.size() - L.first_desc);
                for (int64_t i = 0; i < t; ++i) tmap.push_back(local);
                tiles += t;
                descs.push_back(d);
            }
            L.ndesc = (int64_t)descs.size() - L.first_desc;
            L.total_tiles = tiles;
            L.grid = std::max<int64_t>(1, std::min<int64_t>(tiles, (int64_t)tbl->machine.cu_count *
                                                                       live_blocks_per_cu(tbl->machine, *e)));
            plan->launches.push_back(L);
        }
        plan->ndesc = (int64_t)descs.size();
        const size_t dbytes = descs.size() * sizeof(GroupDesc);
        plan->bytes = dbytes + tmap.size() * sizeof(int32_t);
        if (plan->bytes > 0) {
            hipError_t err = hipSetDevice(tbl->device);
            if (err == hipSuccess) err = hipHostMalloc(&plan->host, plan->bytes, hipHostMallocDefault);
            if (err == hipSuccess) err = hipMalloc(&plan->dev, plan->bytes);
            if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("grouped plan: ") + hipGetErrorString(err));
            std::memcpy(plan->host, descs.data(), dbytes);
            std::memcpy((char *)plan->host + dbytes, tmap.data(), tmap.size() * sizeof(int32_t));
            err = hipMemcpy(plan->dev, plan->host, plan->bytes, hipMemcpyHostToDevice);
            if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("grouped plan upload: ") + hipGetErrorString(err));
        }
        *out = plan.release();
        return PK_OK;
    } catch (const std::exception &ex) {
        return fail(PK_ERR_INVALID_ARG, ex.what());
    }
}

int pk_grouped_plan_run(const pk_grouped_plan *plan, void *hip_stream) {
    if (!plan) return fail(PK_ERR_INVALID_ARG, "null plan");
    const size_t dbytes = (size_t)plan->ndesc * sizeof(GroupDesc);
    for (const auto &L : plan->launches) {
        GroupArgs a;
        a.descs = (const GroupDesc *)plan->dev + L.first_desc;
        a.tile_group = (const int32_t *)((const char *)plan->dev + dbytes) + L.first_tile;
        a.total_tiles = L.total_tiles;
        a.accumulate = plan->accumulate;
        a.pad = 0;
        void *kargs[] = {&a};
        hipError_t err = hipLaunchKernel(L.entry->fn, dim3((unsigned)L.grid), dim3((unsigned)L.entry->threads), kargs,
                                         0, (hipStream_t)hip_stream);
        if (err != hipSuccess)
            return fail(PK_ERR_HIP, std::string("hipLaunchKernel(") + L.entry->name + "): " + hipGetErrorString(err));
    }
    return PK_OK;
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
    if (launches) *launches = (int32_t)plan->launches.size();
    if (total_tiles) {
        int64_t t = 0;
        for (const auto &L : plan->launches) t += L.total_tiles;
        *total_tiles = t;
    }
    if (chosen) {
        if (cap < (int32_t)plan->chosen.size()) return fail(PK_ERR_BUFFER_TOO_SMALL, "cap below the product count");
        std::copy(plan->chosen.begin(), plan->chosen.end(), chosen);
    }
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
