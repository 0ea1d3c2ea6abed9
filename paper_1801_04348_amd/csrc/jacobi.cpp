// Host side of the 1D Jacobi family: launch of the paper's time loop (one
// launch per step, the halves swapping roles), and selection of a leaf and
// its parameters (CASE: streamed bytes over bandwidth with the filled share
// of the last round of tiles; EXHAUSTIVE: HIP-event timing of every feasible
// candidate on a scratch array).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <stdexcept>
#include <vector>

#include "kernels/jacobi.hpp"
#include "pk_internal.hpp"
#include "select.hpp"

namespace pk {

namespace {

int run_steps(const pk_machine &m, const KernelEntry &e, void *a, int64_t N, int64_t steps, size_t elem,
              hipStream_t stream) {
    const int64_t grid = launch_grid(m, e, 1, N - 2);
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

// The several-steps program for a B x S point, if it exists and fits.
const KernelEntry *find_fused(const pk_machine &m, int dtype, int64_t B, int64_t S) {
    for (const auto &e : registry()) {
        if (e.family != PK_FAMILY_JACOBI || e.variant != PK_JACOBI_FUSED || e.dtype != dtype || e.bx != B || e.s != S)
            continue;
        if (e.lds_bytes > m.lds_block || e.threads > m.max_threads_block) return nullptr;
        const KernelResources *r = resources_of(e.name);
        if (!r || regs_per_block(*r, e.threads, m.wave > 0 ? m.wave : 64) > m.regs_block) return nullptr;
        return &e;
    }
    return nullptr;
}

// Steps per launch of the several-steps program for `steps` steps: odd
// counts (after an odd number of steps the state belongs in the other half,
// where the launch writes it) summing to steps - 1, then a last single step,
// so that the last two states are both written, each to its own half.
std::vector<int> fused_plan(int64_t steps) {
    std::vector<int> ks;
    if (steps <= 0) return ks;
    const int64_t R = steps - 1;
    if (R > 0) {
        const int kmax = pkk::kJaMaxSteps - 1;  // odd
        int64_t j = (R + kmax - 1) / kmax;
        if ((j & 1) != (R & 1)) ++j;  // a sum of j odd numbers has j's parity
        std::vector<int64_t> part((size_t)j, 1);
        int64_t left = R - j;  // even; hand out in twos
        for (size_t i = 0; left > 0; i = (i + 1) % part.size())
            if (part[i] + 2 <= kmax) {
                part[i] += 2;
                left -= 2;
            }
        for (int64_t p : part) ks.push_back((int)p);
    }
    ks.push_back(1);
    return ks;
}

int run_fused(const pk_machine &m, const KernelEntry &e, void *a, int64_t N, int64_t steps, size_t elem,
              hipStream_t stream) {
    const int64_t grid = launch_grid(m, e, 1, N - 2);
    char *half[2] = {static_cast<char *>(a), static_cast<char *>(a) + (size_t)N * elem};
    int cur = 0;  // the half holding the current state: the first before step 0
    for (int k : fused_plan(steps)) {
        pkk::JfArgs args{half[cur], half[cur ^ 1], (int32_t)N, k};
        void *kargs[] = {&args};
        hipError_t err = hipLaunchKernel(e.fn, dim3((unsigned)grid), dim3((unsigned)e.threads), kargs, 0, stream);
        if (err != hipSuccess)
            return fail(PK_ERR_HIP, std::string("hipLaunchKernel(") + e.name + "): " + hipGetErrorString(err));
        cur ^= 1;
    }
    return PK_OK;
}

double estimate_fused(const pk_machine &m, const KernelEntry &e, int64_t N, int64_t steps) {
    const int64_t n = std::max<int64_t>(N - 2, 0);
    const int64_t tiles = (n + e.tile_n - 1) / e.tile_n;
    const double clock = m.clock_khz > 0 ? m.clock_khz * 1e3 : 2.4e9;
    double total = 0.0;
    for (int k : fused_plan(steps)) {
        const double halo = (double)(e.tile_n + 2 * k) / e.tile_n;
        const double mem = streaming_seconds(m, e, 4.0 * (double)n * (1.0 + halo), tiles, 4.0 * (e.tile_n + 2 * k),
                                             4.0 * std::min<int64_t>(e.threads, 64));
        // about ten lane operations per point and step, in LDS
        const double alu = 10.0 * k * halo * (double)n / ((double)std::max(m.cu_count, 1) * 64.0 * clock);
        total += std::max(mem, alu + 3e-6);
    }
    return total;
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

int pk_select_jacobi1d(const pk_table *tbl, pk_dtype dtype, int64_t N, int64_t steps, int policy, pk_params *out) {
    if (!tbl || !out) return fail(PK_ERR_INVALID_ARG, "null argument");
    if (dtype != PK_F32 && dtype != PK_I32) return fail(PK_ERR_UNSUPPORTED_DTYPE, "1D Jacobi: f32 or i32");
    if (N < 2 || N > kMaxDim) return fail(PK_ERR_INVALID_ARG, "1D Jacobi needs 2 <= N <= 2^31 - 2^16");
    if (steps < 0) return fail(PK_ERR_INVALID_ARG, "negative step count");
    const int64_t nsteps = std::max<int64_t>(steps, 1);
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
            if (e) c.push_back(C{(int)i, leaf, variant, e, (double)nsteps * estimate_ja(tbl->machine, *e, N)});
        }
        for (size_t i = 0; i < part->fam.points.size(); ++i) {
            const KernelEntry *e = find_fused(tbl->machine, (int)dtype, part->fam.points[i][0], part->fam.points[i][1]);
            if (e) c.push_back(C{(int)i, -1, PK_JACOBI_FUSED, e, estimate_fused(tbl->machine, *e, N, nsteps)});
        }
        if (c.empty()) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no 1D Jacobi leaf holds");
        auto key = std::make_tuple(300 + (int)dtype, N, nsteps, (int64_t)0, policy);
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
                auto go = [&]() {
                    return c[i].leaf < 0 ? run_fused(tbl->machine, *c[i].e, buf, N, nsteps, 4, s)
                                         : run_steps(tbl->machine, *c[i].e, buf, N, nsteps, 4, s);
                };
                if (go() != PK_OK) continue;
                hipEventRecord(e0, s);
                go();
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
        out->variant = c[pick].variant;  // PK_JACOBI_FUSED with leaf -1 for the several-steps program
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
        int rc = pk_select_jacobi1d(tbl, dtype, N, steps, PK_POLICY_CASE, &sel);
        if (rc != PK_OK) return rc;
        params_or_null = &sel;
    }
    if (params_or_null->family != PK_FAMILY_JACOBI) return fail(PK_ERR_INVALID_ARG, "parameters of another family");
    if (params_or_null->variant >= 0 && (params_or_null->variant & PK_JACOBI_FUSED)) {
        if (params_or_null->by != 0 && params_or_null->by != 1) return fail(PK_ERR_INVALID_ARG, "by must be 0 or 1");
        const KernelEntry *e = find_fused(tbl->machine, (int)dtype, params_or_null->bx, params_or_null->s);
        if (!e) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no several-steps instance fits for these parameters");
        return run_fused(tbl->machine, *e, a, N, steps, 4, (hipStream_t)hip_stream);
    }
    pk_params q;
    const KernelEntry *e = nullptr;
    int rc = resolve(tbl, params_or_null, (int)dtype, &q, &e);
    if (rc != PK_OK) return rc;
    return run_steps(tbl->machine, *e, a, N, steps, 4, (hipStream_t)hip_stream);
}

}  // extern "C"
