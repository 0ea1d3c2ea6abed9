// Host side of the matrix-addition family: launch and selection (CASE:
// compulsory bytes over bandwidth with the filled share of the last round of
// tiles; EXHAUSTIVE: HIP-event timing of every feasible candidate).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <stdexcept>

#include "kernels/madd.hpp"
#include "pk_internal.hpp"
#include "select.hpp"

namespace pk {

namespace {

int launch_ma(const pk_machine &m, const KernelEntry &e, const pkk::MaArgs &args, hipStream_t stream) {
    // one workgroup per tile, at most 2^31 - 1 of them (the kernel strides
    // over any tiles beyond)
    const int64_t grid = std::min<int64_t>(launch_grid(m, e, args.M, args.N), 0x7fffffff);
    pkk::MaArgs a = args;
    void *kargs[] = {&a};
    hipError_t err = hipLaunchKernel(e.fn, dim3((unsigned)grid), dim3((unsigned)e.threads), kargs, 0, stream);
    if (err != hipSuccess)
        return fail(PK_ERR_HIP, std::string("hipLaunchKernel(") + e.name + "): " + hipGetErrorString(err));
    return PK_OK;
}

double estimate_ma(const pk_machine &m, const KernelEntry &e, int64_t M, int64_t N) {
    const int64_t tiles = ((M + e.tile_m - 1) / e.tile_m) * ((N + e.tile_n - 1) / e.tile_n);
    // per tile, every work-item issues its S loads of A and of B before adding
    const double inflight = 8.0 * e.tile_m * e.tile_n;
    return streaming_seconds(m, e, 12.0 * (double)M * (double)N, tiles, inflight,
                             4.0 * std::min<int64_t>(e.bx, 64));
}

}  // namespace

}  // namespace pk

using namespace pk;

extern "C" {

int pk_select_madd(const pk_table *tbl, pk_dtype dtype, int64_t M, int64_t N, int policy, pk_params *out) {
    if (!tbl || !out) return fail(PK_ERR_INVALID_ARG, "null argument");
    if (dtype != PK_F32 && dtype != PK_I32) return fail(PK_ERR_UNSUPPORTED_DTYPE, "matrix addition: f32 or i32");
    if (M < 0 || N < 0) return fail(PK_ERR_INVALID_ARG, "negative dimension");
    const pk_table::Part *part = tbl->part(PK_FAMILY_MADD, (int)dtype);
    if (!part || !part->supported) return fail(PK_ERR_UNSUPPORTED_DTYPE, "no matrix-addition table");
    try {
        struct C {
            int point, leaf, variant;
            const KernelEntry *e;
            double est;
        };
        std::vector<C> c;
        for (size_t i = 0; i < part->fam.points.size(); ++i) {
            const int leaf = part->first_leaf[i];
            if (leaf < 0) continue;
            const int variant = (int)part->solved.leaves[leaf].applied;
            const KernelEntry *e = find_instance(PK_FAMILY_MADD, variant, (int)dtype, part->fam.points[i]);
            if (e) c.push_back(C{(int)i, leaf, variant, e, estimate_ma(tbl->machine, *e, M, N)});
        }
        if (c.empty()) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no matrix-addition leaf holds");
        auto key = std::make_tuple(200 + (int)dtype, M, N, (int64_t)0, policy);
        {
            std::lock_guard<std::mutex> g(tbl->cache_mu);
            auto it = tbl->cache.find(key);
            if (it != tbl->cache.end()) {
                *out = it->second;
                return PK_OK;
            }
        }
        int pick = 0;
        if (policy == PK_POLICY_EXHAUSTIVE && M > 0 && N > 0) {
            if (tbl->device < 0) return fail(PK_ERR_INVALID_ARG, "timing needs a table bound to a device");
            if (hipSetDevice(tbl->device) != hipSuccess) return fail(PK_ERR_HIP, "hipSetDevice");
            void *buf = nullptr;
            const size_t bytes = (size_t)M * N * 4;
            if (hipMalloc(&buf, 3 * bytes) != hipSuccess) return fail(PK_ERR_HIP, "timing: allocation failed");
            hipMemset(buf, 0x3c, 2 * bytes);
            hipStream_t s;
            hipEvent_t e0, e1;
            hipStreamCreate(&s);
            hipEventCreate(&e0);
            hipEventCreate(&e1);
            pkk::MaArgs args{buf, (char *)buf + bytes, (char *)buf + 2 * bytes, N, N, N, (int32_t)M, (int32_t)N,
                             N % 4 == 0};
            double best = std::numeric_limits<double>::infinity();
            for (size_t i = 0; i < c.size(); ++i) {
                if (launch_ma(tbl->machine, *c[i].e, args, s) != PK_OK) continue;
                hipEventRecord(e0, s);
                for (int r = 0; r < 3; ++r) launch_ma(tbl->machine, *c[i].e, args, s);
                hipEventRecord(e1, s);
                hipEventSynchronize(e1);
                float ms = 0.f;
                hipEventElapsedTime(&ms, e0, e1);
                if (ms < best) {
                    best = ms;
                    pick = (int)i;
                }
            }
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            hipStreamDestroy(s);
            hipFree(buf);
        } else if (policy == PK_POLICY_CASE || policy == PK_POLICY_EXHAUSTIVE) {
            for (size_t i = 1; i < c.size(); ++i)
                if (c[i].est < c[pick].est) pick = (int)i;
        } else {
            return fail(PK_ERR_INVALID_ARG, "matrix-addition policies: CASE or EXHAUSTIVE");
        }
        point_params(PK_FAMILY_MADD, part->fam.points[c[pick].point], out);
        out->leaf = c[pick].leaf;
        out->variant = c[pick].variant;
        std::lock_guard<std::mutex> g(tbl->cache_mu);
        tbl->cache[key] = *out;
        return PK_OK;
    } catch (const std::exception &ex) {
        return fail(PK_ERR_INVALID_ARG, ex.what());
    }
}

int pk_madd(const pk_table *tbl, const pk_params *params_or_null, pk_dtype dtype, const void *A, int64_t lda,
            const void *B, int64_t ldb, void *C, int64_t ldc, int64_t M, int64_t N, void *hip_stream) {
    if (!tbl) return fail(PK_ERR_INVALID_ARG, "null table");
    if (dtype != PK_F32 && dtype != PK_I32) return fail(PK_ERR_UNSUPPORTED_DTYPE, "matrix addition: f32 or i32");
    if (M < 0 || N < 0 || M > kMaxDim || N > kMaxDim) return fail(PK_ERR_INVALID_ARG, "bad dimension");
    if (M == 0 || N == 0) return PK_OK;
    if (!A || !B || !C || lda < N || ldb < N || ldc < N)
        return fail(PK_ERR_INVALID_ARG, "null pointer or leading dimension too small");
    pk_params sel;
    if (!params_or_null) {
        int rc = pk_select_madd(tbl, dtype, M, N, PK_POLICY_CASE, &sel);
        if (rc != PK_OK) return rc;
        params_or_null = &sel;
    }
    if (params_or_null->family != PK_FAMILY_MADD) return fail(PK_ERR_INVALID_ARG, "parameters of another family");
    pk_params q;
    const KernelEntry *e = nullptr;
    int rc = resolve(tbl, params_or_null, (int)dtype, &q, &e);
    if (rc != PK_OK) return rc;
    const bool vec = ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0) && ((uintptr_t)C % 16 == 0) &&
                     lda % 4 == 0 && ldb % 4 == 0 && ldc % 4 == 0;
    pkk::MaArgs args{A, B, C, lda, ldb, ldc, (int32_t)M, (int32_t)N, vec};
    return launch_ma(tbl->machine, *e, args, (hipStream_t)hip_stream);
}

}  // extern "C"
