// Host side of the 1D Jacobi family: launch of the paper's time loop (one
// launch per step, the halves swapping roles), and selection of a leaf and
// its parameters (CASE: streamed bytes over bandwidth with the filled share
// of the last round of tiles; EXHAUSTIVE: HIP-event timing of every feasible
// candidate on a scratch array).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <stdexcept>

#include "kernels/jacobi.hpp"
#include "pk_internal.hpp"
#include "select.hpp"

namespace pk {

namespace {

int run_steps(const pk_machine &m, const KernelEntry &e, void *a, int64_t N, int64_t steps, size_t elem,
              hipStream_t stream) {
    const int64_t grid = grid_of(m, e, 1, N - 2);
    char *lo = static_cast<char *>(a), *hi = lo + (size_t)N * elem;
    for (int64_t t = 0; t < steps; ++t) {
        // even steps write the second half from the first, odd steps the reverse
        pkk::JaArgs args{t % 2 ? hi : lo, t % 2 ? lo : hi, (int32_t)(N - 2)};
        void *kargs[] = {&args};
        hipError_t err =
            hipLaunchKernel(e.fn, dim3((unsigned)grid), dim3((unsigned)e.threads), kargs, 0, stream);
        if (err != hipSuccess)
            return fail(PK_ERR_HIP, std::string("hipLaunchKernel(") + e.name + "): " + hipGetErrorString(err));
    }
    return PK_OK;
}

double estimate_ja(const pk_machine &m, const KernelEntry &e, int64_t N) {
    const int64_t n = std::max<int64_t>(N - 2, 0);
    const int64_t tiles = (n + e.tile_n - 1) / e.tile_n;
    return streaming_seconds(m, e, 8.0 * (double)n, tiles, 4.0 * (double)(e.tile_n + 2),
                             4.0 * std::min<int64_t>(e.threads, 64));
}

}  // namespace

}  // namespace pk

using namespace pk;

extern "C" {

int pk_select_jacobi1d(const pk_table *tbl, pk_dtype dtype, int64_t N, int policy, pk_params *out) {
    if (!tbl || !out) return fail(PK_ERR_INVALID_ARG, "null argument");
    if (dtype != PK_F32 && dtype != PK_I32) return fail(PK_ERR_UNSUPPORTED_DTYPE, "1D Jacobi: f32 or i32");
    if (N < 2 || N > kMaxDim) return fail(PK_ERR_INVALID_ARG, "1D Jacobi needs 2 <= N <= 2^31 - 2^16");
    const pk_table::Part *part = tbl->part(PK_FAMILY_JACOBI, (int)dtype);
    if (!part || !part->supported) return fail(PK_ERR_UNSUPPORTED_DTYPE, "no 1D Jacobi table");
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
            const KernelEntry *e = find_instance(PK_FAMILY_JACOBI, variant, (int)dtype, part->fam.points[i]);
            if (e) c.push_back(C{(int)i, leaf, variant, e, estimate_ja(tbl->machine, *e, N)});
        }
        if (c.empty()) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no 1D Jacobi leaf holds");
        auto key = std::make_tuple(300 + (int)dtype, N, (int64_t)0, (int64_t)0, policy);
        {
            std::lock_guard<std::mutex> g(tbl->cache_mu);
            auto it = tbl->cache.find(key);
            if (it != tbl->cache.end()) {
                *out = it->second;
                return PK_OK;
            }
        }
        int pick = 0;
        if (policy == PK_POLICY_EXHAUSTIVE && N > 2) {
            if (tbl->device < 0) return fail(PK_ERR_INVALID_ARG, "timing needs a table bound to a device");
            if (hipSetDevice(tbl->device) != hipSuccess) return fail(PK_ERR_HIP, "hipSetDevice");
            void *buf = nullptr;
            if (hipMalloc(&buf, (size_t)N * 8) != hipSuccess) return fail(PK_ERR_HIP, "timing: allocation failed");
            hipMemset(buf, 0, (size_t)N * 8);
            hipStream_t s;
            hipEvent_t e0, e1;
            hipStreamCreate(&s);
            hipEventCreate(&e0);
            hipEventCreate(&e1);
            double best = std::numeric_limits<double>::infinity();
            for (size_t i = 0; i < c.size(); ++i) {
                if (run_steps(tbl->machine, *c[i].e, buf, N, 2, 4, s) != PK_OK) continue;
                hipEventRecord(e0, s);
                run_steps(tbl->machine, *c[i].e, buf, N, 4, 4, s);
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
            return fail(PK_ERR_INVALID_ARG, "1D Jacobi policies: CASE or EXHAUSTIVE");
        }
        point_params(PK_FAMILY_JACOBI, part->fam.points[c[pick].point], out);
        out->leaf = c[pick].leaf;
        out->variant = c[pick].variant;
        std::lock_guard<std::mutex> g(tbl->cache_mu);
        tbl->cache[key] = *out;
        return PK_OK;
    } catch (const std::exception &ex) {
        return fail(PK_ERR_INVALID_ARG, ex.what());
    }
}

int pk_jacobi1d(const pk_table *tbl, const pk_params *params_or_null, pk_dtype dtype, void *a, int64_t N,
                int64_t steps, void *hip_stream) {
    if (!tbl) return fail(PK_ERR_INVALID_ARG, "null table");
    if (dtype != PK_F32 && dtype != PK_I32) return fail(PK_ERR_UNSUPPORTED_DTYPE, "1D Jacobi: f32 or i32");
    if (N < 2 || N > kMaxDim || steps < 0) return fail(PK_ERR_INVALID_ARG, "1D Jacobi needs 2 <= N <= 2^31 - 2^16, steps >= 0");
    if (N == 2 || steps == 0) return PK_OK;
    if (!a) return fail(PK_ERR_INVALID_ARG, "null array");
    pk_params sel;
    if (!params_or_null) {
        int rc = pk_select_jacobi1d(tbl, dtype, N, PK_POLICY_CASE, &sel);
        if (rc != PK_OK) return rc;
        params_or_null = &sel;
    }
    if (params_or_null->family != PK_FAMILY_JACOBI) return fail(PK_ERR_INVALID_ARG, "parameters of another family");
    pk_params q;
    const KernelEntry *e = nullptr;
    int rc = resolve(tbl, params_or_null, (int)dtype, &q, &e);
    if (rc != PK_OK) return rc;
    return run_steps(tbl->machine, *e, a, N, steps, 4, (hipStream_t)hip_stream);
}

}  // extern "C"
