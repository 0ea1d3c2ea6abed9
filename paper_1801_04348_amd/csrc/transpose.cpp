// Host side of the transposition family: launch, and selection of a leaf and
// its parameters (CASE: bytes over bandwidth by program, with the share of
// the last round of tiles that is filled; EXHAUSTIVE: HIP-event timing of every
// feasible candidate on scratch buffers).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <stdexcept>

#include "kernels/transpose.hpp"
#include "pk_internal.hpp"
#include "select.hpp"

namespace pk {

namespace {

int launch_tr(const pk_machine &m, const KernelEntry &e, const pkk::TrArgs &args, hipStream_t stream) {
    const int64_t grid = launch_grid(m, e, args.M, args.N);
    pkk::TrArgs a = args;
    void *kargs[] = {&a};
    hipError_t err = hipLaunchKernel(e.fn, dim3((unsigned)grid), dim3((unsigned)e.threads), kargs, 0, stream);
    if (err != hipSuccess)
        return fail(PK_ERR_HIP, std::string("hipLaunchKernel(") + e.name + "): " + hipGetErrorString(err));
    return PK_OK;
}

double estimate_tr(const pk_machine &m, const KernelEntry &e, int64_t M, int64_t N) {
    const int64_t tiles = ((M + e.tile_m - 1) / e.tile_m) * ((N + e.tile_n - 1) / e.tile_n);
    // reads run along rows of A (bx elements); the cached program writes
    // along rows of C (by * s elements), the direct one 4-byte strided
    const double rd = 4.0 * std::min<int64_t>(e.bx, 64);
    const double wr = (e.variant & PK_VALU_NOLDS) ? 4.0 : 4.0 * std::min<int64_t>(e.tile_m, 64);
    return streaming_seconds(m, e, 8.0 * (double)M * (double)N, tiles, 4.0 * e.tile_m * e.tile_n,
                             std::min(rd, wr));
}

struct TrCand {
    int point, leaf, variant;
    const KernelEntry *entry;
    double est;
};

std::vector<TrCand> tr_feasible(const pk_table *tbl, int dtype, int64_t M, int64_t N) {
    std::vector<TrCand> out;
    const pk_table::Part *part = tbl->part(PK_FAMILY_TRANSPOSE, dtype);
    if (!part || !part->supported) return out;
    for (size_t i = 0; i < part->fam.points.size(); ++i) {
        const int leaf = part->first_leaf[i];
        if (leaf < 0) continue;
        const int variant = (int)part->solved.leaves[leaf].applied;
        const KernelEntry *e = find_instance(PK_FAMILY_TRANSPOSE, variant, dtype, part->fam.points[i]);
        if (!e) continue;
        out.push_back(TrCand{(int)i, leaf, variant, e, estimate_tr(tbl->machine, *e, M, N)});
    }
    return out;
}

}  // namespace

}  // namespace pk

using namespace pk;

extern "C" {

int pk_select_transpose(const pk_table *tbl, pk_dtype dtype, int64_t M, int64_t N, int policy, pk_params *out) {
    if (!tbl || !out) return fail(PK_ERR_INVALID_ARG, "null argument");
    if (dtype != PK_F32 && dtype != PK_I32) return fail(PK_ERR_UNSUPPORTED_DTYPE, "transposition: 4-byte elements");
    if (M < 0 || N < 0) return fail(PK_ERR_INVALID_ARG, "negative dimension");
    try {
        std::vector<TrCand> c = tr_feasible(tbl, (int)dtype, M, N);
        if (c.empty()) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no transposition leaf holds");
        auto key = std::make_tuple(100 + (int)dtype, M, N, (int64_t)0, policy);
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
            void *A = nullptr, *C = nullptr;
            const size_t bytes = (size_t)M * N * 4;
            if (hipMalloc(&A, bytes) != hipSuccess || hipMalloc(&C, bytes) != hipSuccess) {
                hipFree(A);
                return fail(PK_ERR_HIP, "timing: allocation failed");
            }
            hipMemset(A, 0x3c, bytes);
            hipStream_t s;
            hipEvent_t e0, e1;
            hipStreamCreate(&s);
            hipEventCreate(&e0);
            hipEventCreate(&e1);
            pkk::TrArgs args{A, C, N, M, (int32_t)M, (int32_t)N};
            double best = std::numeric_limits<double>::infinity();
            for (size_t i = 0; i < c.size(); ++i) {
                if (launch_tr(tbl->machine, *c[i].entry, args, s) != PK_OK) continue;
                hipEventRecord(e0, s);
                for (int r = 0; r < 3; ++r) launch_tr(tbl->machine, *c[i].entry, args, s);
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
            hipFree(A);
            hipFree(C);
        } else if (policy == PK_POLICY_CASE || policy == PK_POLICY_EXHAUSTIVE) {
            for (size_t i = 1; i < c.size(); ++i)
                if (c[i].est < c[pick].est) pick = (int)i;
        } else {
            return fail(PK_ERR_INVALID_ARG, "transposition policies: CASE or EXHAUSTIVE");
        }
        const pk_table::Part *part = tbl->part(PK_FAMILY_TRANSPOSE, (int)dtype);
        point_params(PK_FAMILY_TRANSPOSE, part->fam.points[c[pick].point], out);
        out->leaf = c[pick].leaf;
        out->variant = c[pick].variant;
        std::lock_guard<std::mutex> g(tbl->cache_mu);
        tbl->cache[key] = *out;
        return PK_OK;
    } catch (const std::exception &ex) {
        return fail(PK_ERR_INVALID_ARG, ex.what());
    }
}

int pk_transpose(const pk_table *tbl, const pk_params *params_or_null, pk_dtype dtype, const void *A, int64_t lda,
                 void *C, int64_t ldc, int64_t M, int64_t N, void *hip_stream) {
    if (!tbl) return fail(PK_ERR_INVALID_ARG, "null table");
    if (dtype != PK_F32 && dtype != PK_I32) return fail(PK_ERR_UNSUPPORTED_DTYPE, "transposition: 4-byte elements");
    if (M < 0 || N < 0 || M > kMaxDim || N > kMaxDim) return fail(PK_ERR_INVALID_ARG, "bad dimension");
    if (M == 0 || N == 0) return PK_OK;
    if (!A || !C || lda < N || ldc < M) return fail(PK_ERR_INVALID_ARG, "null pointer or leading dimension too small");
    pk_params sel;
    if (!params_or_null) {
        int rc = pk_select_transpose(tbl, dtype, M, N, PK_POLICY_CASE, &sel);
        if (rc != PK_OK) return rc;
        params_or_null = &sel;
    }
    if (params_or_null->family != PK_FAMILY_TRANSPOSE)
        return fail(PK_ERR_INVALID_ARG, "parameters of another family");
    pk_params q;
    const KernelEntry *e = nullptr;
    int rc = resolve(tbl, params_or_null, (int)dtype, &q, &e);
    if (rc != PK_OK) return rc;
    pkk::TrArgs args{A, C, lda, ldc, (int32_t)M, (int32_t)N};
    return launch_tr(tbl->machine, *e, args, (hipStream_t)hip_stream);
}

}  // extern "C"
