// Host side of the polynomial-division family: the figure's while loop as one
// launch per step, a final clear of the eliminated coefficients, and
// selection of a leaf and its parameters (CASE: streamed bytes per step with
// the per-launch latency; EXHAUSTIVE: HIP-event timing of every feasible
// candidate on a scratch problem of the same sizes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <stdexcept>

#include "kernels/polydiv.hpp"
#include "pk_internal.hpp"
#include "select.hpp"

namespace pk {

namespace {

__global__ void pd_clear(uint32_t *__restrict__ a, int64_t lo, int64_t hi) {
    for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0u;
}

uint64_t barrett_mu(uint32_t P) { return (uint64_t)((((unsigned __int128)1) << 64) / P); }

int run_division(const pk_machine &m, const KernelEntry &e, uint32_t *a, int64_t N, const uint32_t *b, int64_t M,
                 uint32_t P, hipStream_t stream) {
    if (N <= M) return PK_OK;
    const int64_t grid = launch_grid(m, e, 1, M);
    pkk::PdArgs g{a, b, (int32_t)M, 0, P, barrett_mu(P)};
    for (int64_t n = N; n - 1 >= M; --n) {
        g.n = (int32_t)n;
        void *kargs[] = {&g};
        hipError_t err = hipLaunchKernel(e.fn, dim3((unsigned)grid), dim3((unsigned)e.threads), kargs, 0, stream);
        if (err != hipSuccess)
            return fail(PK_ERR_HIP, std::string("hipLaunchKernel(") + e.name + "): " + hipGetErrorString(err));
    }
    const int64_t span = N - M;
    const unsigned cg = (unsigned)std::min<int64_t>((span + 255) / 256, 1024);
    hipLaunchKernelGGL(pd_clear, dim3(cg), dim3(256), 0, stream, a, M, N);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("pd_clear: ") + hipGetErrorString(err));
    return PK_OK;
}

// The one-launch program (kernels/polydiv.hpp, polydiv_fused) for a B x S
// point and K = N - M quotient coefficients: the instance whose register
// slots hold K, if it exists and fits the machine.
const KernelEntry *find_fused(const pk_machine &m, int64_t B, int64_t S, int64_t K) {
    if (K < 1 || K > pkk::kPdMaxK) return nullptr;
    const int variant = PK_POLYDIV_FUSED | (K > 128 ? PK_POLYDIV_WIDE : 0);
    for (const auto &e : registry()) {
        if (e.family != PK_FAMILY_POLYDIV || e.variant != variant || e.bx != B || e.s != S) continue;
        if (e.lds_bytes > m.lds_block || e.threads > m.max_threads_block) return nullptr;
        const KernelResources *r = resources_of(e.name);
        if (!r || regs_per_block(*r, e.threads, m.wave > 0 ? m.wave : 64) > m.regs_block) return nullptr;
        return &e;
    }
    return nullptr;
}

int run_fused(const pk_machine &m, const KernelEntry &e, uint32_t *a, int64_t N, const uint32_t *b, int64_t M,
              uint32_t P, hipStream_t stream) {
    if (N <= M) return PK_OK;
    const int64_t grid = launch_grid(m, e, 1, M);
    pkk::PdArgs g{a, b, (int32_t)M, (int32_t)N, P, barrett_mu(P)};
    void *kargs[] = {&g};
    hipError_t err = hipLaunchKernel(e.fn, dim3((unsigned)grid), dim3((unsigned)e.threads), kargs, 0, stream);
    if (err != hipSuccess)
        return fail(PK_ERR_HIP, std::string("hipLaunchKernel(") + e.name + "): " + hipGetErrorString(err));
    const int64_t span = N - M;
    const unsigned cg = (unsigned)std::min<int64_t>((span + 255) / 256, 1024);
    hipLaunchKernelGGL(pd_clear, dim3(cg), dim3(256), 0, stream, a, M, N);
    err = hipGetLastError();
    if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("pd_clear: ") + hipGetErrorString(err));
    return PK_OK;
}

double estimate_fused(const pk_machine &m, const KernelEntry &e, int64_t N, int64_t M) {
    const double K = (double)(N - M);
    const double clock = m.clock_khz > 0 ? m.clock_khz * 1e3 : 2.4e9;
    // phase 1: a dependent chain of K steps, each a lane read, a product
    // reduction and the register-slot updates of one wavefront
    const double slots = (e.variant & PK_POLYDIV_WIDE) ? 16.0 : 2.0;
    const double phase1 = K * (160.0 + 60.0 * slots) / clock;
    // phase 2: K reduced products per remainder coefficient, about 16 VALU
    // instructions each, over the resident lanes
    const int64_t tiles = (M + e.tile_n - 1) / e.tile_n;
    const double lanes = (double)std::min<int64_t>(tiles, (int64_t)m.cu_count * blocks_per_cu(m, e)) * e.threads;
    const double lane_rate = std::min(lanes, (double)m.cu_count * 64.0 * 4.0) * clock / 4.0;
    const double phase2 = (double)M * K * 16.0 / std::max(lane_rate, 1.0);
    return phase1 + phase2 + 6e-6;
}

double estimate_pd(const pk_machine &m, const KernelEntry &e, int64_t N, int64_t M) {
    if (N <= M) return 0.0;
    const int64_t tiles = (M + e.tile_n - 1) / e.tile_n;
    // a step reads a and b and writes a over M coefficients
    const double step = streaming_seconds(m, e, 12.0 * (double)M, tiles, 8.0 * (double)e.tile_n,
                                          4.0 * std::min<int64_t>(e.threads, 64));
    return (double)(N - M) * step;
}

int check_args(int64_t N, int64_t M, uint32_t P) {
    if (N < 0 || M < 1 || N > kMaxDim || M > kMaxDim)
        return fail(PK_ERR_INVALID_ARG, "polynomial division needs N >= 0, M >= 1, both at most 2^31 - 2^16");
    if (P < 2 || P >= 0x80000000u) return fail(PK_ERR_INVALID_ARG, "modulus P must satisfy 2 <= P < 2^31");
    return PK_OK;
}

}  // namespace

}  // namespace pk

using namespace pk;

extern "C" {

int pk_select_polydiv(const pk_table *tbl, int64_t N, int64_t M, int policy, pk_params *out) {
    if (!tbl || !out) return fail(PK_ERR_INVALID_ARG, "null argument");
    int rc = check_args(N, M, 2);
    if (rc != PK_OK) return rc;
    const pk_table::Part *part = tbl->part(PK_FAMILY_POLYDIV, PK_I32);
    if (!part || !part->supported) return fail(PK_ERR_UNSUPPORTED_DTYPE, "no polynomial-division table");
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
            const KernelEntry *e = find_instance(PK_FAMILY_POLYDIV, variant, PK_I32, part->fam.points[i]);
            if (e) c.push_back(C{(int)i, leaf, variant, e, estimate_pd(tbl->machine, *e, N, M)});
        }
        for (size_t i = 0; i < part->fam.points.size(); ++i) {
            const auto &pt = part->fam.points[i];
            const KernelEntry *e = find_fused(tbl->machine, pt[0], pt[1], N - M);
            if (e) c.push_back(C{(int)i, -1, PK_POLYDIV_FUSED, e, estimate_fused(tbl->machine, *e, N, M)});
        }
        if (c.empty()) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no polynomial-division leaf holds");
        auto key = std::make_tuple(400, N, M, (int64_t)0, policy);
        {
            std::lock_guard<std::mutex> g(tbl->cache_mu);
            auto it = tbl->cache.find(key);
            if (it != tbl->cache.end()) {
                *out = it->second;
                return PK_OK;
            }
        }
        int pick = 0;
        if (policy == PK_POLICY_EXHAUSTIVE && N > M) {
            if (tbl->device < 0) return fail(PK_ERR_INVALID_ARG, "timing needs a table bound to a device");
            if (hipSetDevice(tbl->device) != hipSuccess) return fail(PK_ERR_HIP, "hipSetDevice");
            void *buf = nullptr;
            if (hipMalloc(&buf, (size_t)(N + M) * 4) != hipSuccess)
                return fail(PK_ERR_HIP, "timing: allocation failed");
            hipMemset(buf, 0, (size_t)(N + M) * 4);
            uint32_t *a = static_cast<uint32_t *>(buf), *b = a + N;
            hipStream_t s;
            hipEvent_t e0, e1;
            hipStreamCreate(&s);
            hipEventCreate(&e0);
            hipEventCreate(&e1);
            double best = std::numeric_limits<double>::infinity();
            for (size_t i = 0; i < c.size(); ++i) {
                auto go = [&]() {
                    return c[i].leaf < 0 ? run_fused(tbl->machine, *c[i].e, a, N, b, M, 65521u, s)
                                         : run_division(tbl->machine, *c[i].e, a, N, b, M, 65521u, s);
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
            return fail(PK_ERR_INVALID_ARG, "polynomial-division policies: CASE or EXHAUSTIVE");
        }
        point_params(PK_FAMILY_POLYDIV, part->fam.points[c[pick].point], out);
        out->leaf = c[pick].leaf;
        out->variant = c[pick].leaf < 0 ? c[pick].e->variant : c[pick].variant;
        std::lock_guard<std::mutex> g(tbl->cache_mu);
        tbl->cache[key] = *out;
        return PK_OK;
    } catch (const std::exception &ex) {
        return fail(PK_ERR_INVALID_ARG, ex.what());
    }
}

int pk_polydiv(const pk_table *tbl, const pk_params *params_or_null, uint32_t *a, int64_t N, const uint32_t *b,
               int64_t M, uint32_t P, void *hip_stream) {
    if (!tbl) return fail(PK_ERR_INVALID_ARG, "null table");
    int rc = check_args(N, M, P);
    if (rc != PK_OK) return rc;
    if (N <= M) return PK_OK;
    if (!a || !b) return fail(PK_ERR_INVALID_ARG, "null array");
    pk_params sel;
    if (!params_or_null) {
        rc = pk_select_polydiv(tbl, N, M, PK_POLICY_CASE, &sel);
        if (rc != PK_OK) return rc;
        params_or_null = &sel;
    }
    if (params_or_null->family != PK_FAMILY_POLYDIV) return fail(PK_ERR_INVALID_ARG, "parameters of another family");
    if (params_or_null->variant >= 0 && (params_or_null->variant & PK_POLYDIV_FUSED)) {
        if (N - M > pkk::kPdMaxK) return fail(PK_ERR_INVALID_ARG, "one-launch division needs N - M <= 1024");
        const KernelEntry *e = find_fused(tbl->machine, params_or_null->bx, params_or_null->s, N - M);
        if (!e) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no one-launch division instance fits for these parameters");
        return run_fused(tbl->machine, *e, a, N, b, M, P, (hipStream_t)hip_stream);
    }
    pk_params q;
    const KernelEntry *e = nullptr;
    rc = resolve(tbl, params_or_null, PK_I32, &q, &e);
    if (rc != PK_OK) return rc;
    return run_division(tbl->machine, *e, a, N, b, M, P, (hipStream_t)hip_stream);
}

}  // extern "C"
