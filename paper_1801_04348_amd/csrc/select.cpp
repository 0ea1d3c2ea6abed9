// Selection policies over the feasible set F = {(leaf, E) : the leaf's system
// holds at the bound machine and at E, and an instance of its program exists}.
//
// CASE: the paper fixes the leaf for given parameters by the case discussion
// and leaves the program parameters to auto-tuning (Section 1); here they are
// chosen by an analytic estimate of the launch time:
//   tiles     = ceil(M / tile_m) * ceil(N / tile_n)
//   occupancy = workgroups resident per compute unit (LDS, registers, threads,
//               workgroup slots)
//   rounds    = ceil(tiles / (compute units * occupancy))
//   compute   = rounds * occupancy * 2 * tile_m * tile_n * K / (rate * clock)
//               with rate the per-CU throughput of the program's inner loop
//               (matrix cores, or VALU limited by LDS reads per FMA)
//   traffic   = bytes the tiles read (each tile reads its A and B panels),
//               over an on-chip cache bandwidth, and compulsory bytes over HBM
//   estimate  = max(compute, traffic) + a fixed launch cost
// EXHAUSTIVE: every candidate is timed with HIP events on the device and the
// fastest kept (cached per shape).
#include "select.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <stdexcept>

namespace pk {

namespace {
constexpr double kLaunchSeconds = 4e-6;
constexpr double kCacheBytesPerSecond = 12e12;  // aggregate L2/MALL read rate used by the estimate
constexpr double kHbmBytesPerSecond = 8e12;

int elem_bytes(int dtype) { return dtype == PK_BF16 ? 2 : 4; }

// multiply-accumulate throughput of one compute unit, flop per clock
double cu_rate(const pk_machine &m, const KernelEntry &e, int dtype) {
    const int threads = e.threads;
    const int wave = m.wave > 0 ? m.wave : 64;
    const double lanes = (double)threads / (double)(wave * ((threads + wave - 1) / wave));
    if (e.family == PK_FAMILY_MFMA) return dtype == PK_BF16 ? 2048.0 : 256.0;
    // VALU: 64 lanes x 4 SIMDs / 4 cycles = 64 multiply-adds per clock for
    // float32; int32 multiplies run at a quarter of that.  The tiled kernel
    // also reads 1 + s LDS words per s multiply-adds (32 words per clock).
    const double s = std::max(1, (e.variant & PK_VALU_NOLDS) ? 1 : e.s);
    double mads = dtype == PK_I32 ? 16.0 : 64.0;
    if (!(e.variant & PK_VALU_NOLDS)) mads = std::min(mads, 32.0 * s / (1.0 + s));
    else mads = std::min(mads, 16.0);  // global/L1 bound
    return 2.0 * mads * lanes;
}
}  // namespace

double estimate_seconds(const pk_machine &m, const KernelEntry &e, int dtype, int64_t M, int64_t N, int64_t K) {
    const double clock = (m.clock_khz > 0 ? m.clock_khz : 2400000) * 1e3;
    const int64_t tm = (M + e.tile_m - 1) / e.tile_m, tn = (N + e.tile_n - 1) / e.tile_n;
    const int64_t tiles = tm * tn;
    const int64_t occ = blocks_per_cu(m, e);
    const int64_t slots = (int64_t)m.cu_count * occ;
    const int64_t rounds = (tiles + slots - 1) / slots;
    const double flops_tile = 2.0 * e.tile_m * e.tile_n * (double)std::max<int64_t>(K, 1);
    const double compute = rounds * occ * flops_tile / (cu_rate(m, e, dtype) * clock);
    const double es = elem_bytes(dtype);
    const double tile_bytes = es * (double)tiles * (double)K * (e.tile_m + e.tile_n);
    const double out_bytes = 4.0 * (double)M * N;
    const double hbm = (es * ((double)M * K + (double)K * N) + out_bytes) / kHbmBytesPerSecond;
    const double traffic = std::max(tile_bytes / kCacheBytesPerSecond, hbm);
    return std::max(compute, traffic) + kLaunchSeconds;
}

void fill_params(const pk_table *tbl, const Candidate &c, int dtype, pk_params *out) {
    const pk_table::Part *part = tbl->part(c.family, dtype);
    point_params(c.family, part->fam.points[c.point], out);
    out->leaf = c.leaf;
    out->variant = c.variant;
}

std::vector<Candidate> feasible(const pk_table *tbl, int dtype, int64_t M, int64_t N, int64_t K, const void *A,
                                int64_t lda, const void *B, int64_t ldb) {
    std::vector<Candidate> out;
    for (int family = 0; family < PK_NUM_FAMILIES; ++family) {
        const pk_table::Part *part = tbl->part(family, dtype);
        if (!part || !part->supported) continue;
        if (A && !data_ok(family, dtype, A, lda, B, ldb)) continue;
        for (size_t i = 0; i < part->fam.points.size(); ++i) {
            const int leaf = part->first_leaf[i];
            if (leaf < 0) continue;
            Candidate c;
            c.family = family;
            c.point = (int)i;
            c.leaf = leaf;
            c.variant = (int)part->solved.leaves[leaf].applied;
            c.entry = find_instance(family, c.variant, dtype, part->fam.points[i]);
            if (!c.entry) continue;
            c.estimate = estimate_seconds(tbl->machine, *c.entry, dtype, M, N, K);
            out.push_back(c);
        }
    }
    return out;
}

namespace {

// Times every candidate on the table's device; returns the index of the fastest.
int time_candidates(const pk_table *tbl, int dtype, int64_t M, int64_t N, int64_t K,
                    const std::vector<Candidate> &cands, std::vector<double> *secs) {
    if (tbl->device < 0) throw std::runtime_error("exhaustive selection needs a table bound to a device");
    hipError_t err = hipSetDevice(tbl->device);
    if (err != hipSuccess) throw std::runtime_error(std::string("hipSetDevice: ") + hipGetErrorString(err));
    const size_t es = dtype == PK_BF16 ? 2 : 4;
    void *A = nullptr, *B = nullptr, *C = nullptr;
    const size_t bA = std::max<size_t>(es * M * K, 16), bB = std::max<size_t>(es * K * N, 16),
                 bC = std::max<size_t>(4 * M * N, 16);
    if (hipMalloc(&A, bA) != hipSuccess || hipMalloc(&B, bB) != hipSuccess || hipMalloc(&C, bC) != hipSuccess) {
        hipFree(A);
        hipFree(B);
        throw std::runtime_error("exhaustive selection: device allocation failed");
    }
    hipMemset(A, 0, bA);
    hipMemset(B, 0, bB);
    hipStream_t s;
    hipEvent_t e0, e1;
    hipStreamCreate(&s);
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    int best = -1;
    double best_t = std::numeric_limits<double>::infinity();
    secs->assign(cands.size(), std::numeric_limits<double>::infinity());
    MmArgs args{A, B, C, K, N, N, (int32_t)M, (int32_t)N, (int32_t)K, 0};
    for (size_t i = 0; i < cands.size(); ++i) {
        const KernelEntry &e = *cands[i].entry;
        if (launch(tbl->machine, e, args, s) != PK_OK) continue;  // warm-up
        hipEventRecord(e0, s);
        int reps = 0;
        float ms = 0.f;
        // at least 3 launches, up to about 20 ms of work
        do {
            launch(tbl->machine, e, args, s);
            ++reps;
            if (reps == 3 || reps % 8 == 0) {
                hipEventRecord(e1, s);
                hipEventSynchronize(e1);
                hipEventElapsedTime(&ms, e0, e1);
            }
        } while (reps < 3 || (ms < 20.f && reps < 200));
        const double t = ms * 1e-3 / reps;
        (*secs)[i] = t;
        if (t < best_t) {
            best_t = t;
            best = (int)i;
        }
    }
    hipStreamSynchronize(s);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipStreamDestroy(s);
    hipFree(A);
    hipFree(B);
    hipFree(C);
    return best;
}

}  // namespace

int select_params(const pk_table *tbl, int dtype, int64_t M, int64_t N, int64_t K, int policy, bool cache,
                  pk_params *out, const void *A, int64_t lda, const void *B, int64_t ldb) {
    std::vector<Candidate> cands = feasible(tbl, dtype, M, N, K, A, lda, B, ldb);
    if (cands.empty()) return fail(PK_ERR_NO_FEASIBLE_BRANCH, "no leaf of the case table holds for this dtype");
    const bool aligned_any = A == nullptr;
    auto key = std::make_tuple(dtype, M, N, K, policy);
    if (cache && aligned_any) {
        std::lock_guard<std::mutex> g(tbl->cache_mu);
        auto it = tbl->cache.find(key);
        if (it != tbl->cache.end()) {
            *out = it->second;
            return PK_OK;
        }
    }
    int pick = 0;
    if (policy == PK_POLICY_CASE || policy == PK_POLICY_LEARNED) {
        for (size_t i = 1; i < cands.size(); ++i)
            if (cands[i].estimate < cands[pick].estimate) pick = (int)i;
        fill_params(tbl, cands[pick], dtype, out);
        if (policy == PK_POLICY_LEARNED) return fail(PK_ERR_COST_MODEL, "no cost model loaded; CASE pick returned");
    } else if (policy == PK_POLICY_EXHAUSTIVE) {
        std::vector<double> secs;
        pick = time_candidates(tbl, dtype, M, N, K, cands, &secs);
        if (pick < 0) return fail(PK_ERR_HIP, "no candidate could be launched");
        fill_params(tbl, cands[pick], dtype, out);
    } else {
        return fail(PK_ERR_INVALID_ARG, "unknown policy");
    }
    if (cache && aligned_any) {
        std::lock_guard<std::mutex> g(tbl->cache_mu);
        tbl->cache[key] = *out;
    }
    return PK_OK;
}

}  // namespace pk
