// Selection policies over the feasible set F = {(leaf, E) : the leaf's system
// holds at the bound machine and at E, and an instance of its program exists}.
//
// CASE: the paper fixes the leaf for given parameters by the case discussion
// and leaves the program parameters to auto-tuning (Section 1); here they are
// chosen by an analytic estimate of the launch time:
//   tiles     = ceil(M / tile_m) * ceil(N / tile_n)
//   occupancy = workgroups resident per compute unit (LDS, registers, threads,
//               workgroup slots, as the bound machine reports them)
//   rounds    = ceil(tiles / (compute units * occupancy))
//   per round = max(occupancy * 2 * tile_m * tile_n * K / (rate * eff * clock),
//                   K steps * step latency)
//               rate: per-CU throughput of the program's inner loop (matrix
//               cores; or VALU multiply-adds limited by the LDS words read per
//               multiply-add); eff: the share of that rate a tile sustains,
//               falling with the LDS/L2 words moved per flop, 1/tile_m +
//               1/tile_n; step latency: one global-load round trip plus the
//               barriers of a K step, hidden in part by a second LDS stage
//   traffic   = bytes the tiles read (each tile reads its A and B panels) over
//               an on-chip cache bandwidth, and compulsory bytes over HBM
//   estimate  = max(rounds * per round, traffic) + a fixed launch cost
// The constants (eff's shape, step latencies) were set from event timings of
// these kernels on gfx950; the estimate only has to rank candidates.
// EXHAUSTIVE: every candidate is launched and timed with HIP events on the
// device (back-to-back launches, mean), the least CASE estimate first; a
// candidate whose first three launches are already 1.5x slower than the best
// so far is not timed further, nor one whose single warm-up launch takes over
// a millisecond and twice the best.  The fastest is kept (cached per shape).
#include "select.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <stdexcept>

namespace pk {

namespace {
constexpr double kLaunchSeconds = 4e-6;
constexpr double kHbmBytesPerSecond = 8e12;
constexpr double kAtomicAddsPerSecond = 4e11;  // float atomic additions to C, whole device

int elem_bytes(int dtype) { return dtype == PK_BF16 ? 2 : 4; }

// multiply-accumulate throughput of one compute unit, flop per clock
double cu_rate(const pk_machine &m, const KernelEntry &e, int dtype) {
    const int threads = e.threads;
    const int wave = m.wave > 0 ? m.wave : 64;
    const double lanes = (double)threads / (double)(wave * ((threads + wave - 1) / wave));
    // MFMA: float32 256, bfloat16 2048; int32 on the int8 matrix cores 8192
    // int8 operations per clock, ten int8 products per int32 one
    if (e.family == PK_FAMILY_MFMA) return dtype == PK_BF16 ? 2048.0 : dtype == PK_I32 ? 819.2 : 256.0;
    // VALU: 64 lanes x 4 SIMDs / 4 cycles = 64 multiply-adds per clock for
    // float32; int32 multiply-adds run at half of that (measured).  The tiled kernel
    // also reads 1 + s LDS words per s multiply-adds, which caps it near 24
    // multiply-adds per clock, rising slowly with s; the direct kernel is
    // bound by global/L1 reads (about one multiply-add per clock).
    // int32 (fitted on the timings of every feasible candidate of 200 random
    // int32 shapes, 140 to fit and 60 to check): the tiled kernel's relative
    // rates 0.85, 0.9, 0.5, 0.7 for s = 1, 2, 4, 8 of the 32 multiply-adds
    // per clock; the 2-D micro-tile program (four k of A and s columns of B
    // per LDS read) up to 1.1 times that, or about 36 LDS words per clock.
    const double s = std::max(1, e.s);
    double mads = dtype == PK_I32 ? 32.0 : 64.0;
    if (e.family == PK_FAMILY_VALU2) {
        // 2-D micro-tiles: (s + sy) / (s sy) LDS words per multiply-add
        // against the LDS's words per clock, up to the ALU rate
        const double sy = std::max(1, e.sy);
        if (dtype == PK_I32) return 2.0 * lanes * std::min(mads * 1.1, 36.0 * s * sy / (s + sy));
        return 2.0 * lanes * std::min(mads, 24.0 * s * sy / (s + sy));
    }
    if (e.variant & PK_VALU_NOLDS)
        mads = 1.0;
    else if (dtype == PK_I32)
        mads *= e.s <= 1 ? 0.85 : e.s == 2 ? 0.9 : e.s <= 4 ? 0.5 : 0.70;
    else
        mads = std::min(mads, 24.0 * std::pow(s / (1.0 + s), 0.25));
    return 2.0 * mads * lanes;
}
}  // namespace

double streaming_seconds(const pk_machine &m, const KernelEntry &e, double bytes, int64_t tiles,
                         double inflight_bytes_per_tile, double segment_bytes) {
    const int64_t ncu = std::max<int32_t>(m.cu_count, 1);
    const int64_t bpc = blocks_per_cu(m, e);
    tiles = std::max<int64_t>(tiles, 1);
    const int64_t per_cu = (tiles + ncu - 1) / ncu;  // tiles of the busiest compute unit
    const int64_t active = std::min(ncu, tiles);
    const double imbalance = (double)(per_cu * ncu) / (double)tiles;
    const double resident = (double)std::min(bpc, per_cu);
    const double inflight = std::min(1.0, resident * inflight_bytes_per_tile / 65536.0);
    // a wavefront's access is 64 lanes x 4 bytes: runs along a row shorter
    // than 256 bytes split it over several rows (transposition of order 2^14:
    // the 128-byte runs of 32-wide tiles 4.4 TB/s, the 256-byte ones 4.9)
    const double seg = std::min(1.0, segment_bytes / 256.0);
    // one compute unit alone draws about 64 GB/s; all of them, 8 TB/s
    const double bw = std::min(8e12, 64e9 * (double)active) * 0.85 * std::max(inflight * seg, 1e-3);
    const double rounds = (double)((per_cu + bpc - 1) / bpc);
    return bytes * (tiles >= ncu ? imbalance : 1.0) / bw + 0.5e-6 * rounds + 3e-6;
}

std::vector<int> k_splits(const pk_machine &m, const KernelEntry &e, int64_t M, int64_t N, int64_t K) {
    std::vector<int> out;
    if (e.family != PK_FAMILY_MFMA || e.bk <= 0 || !split_twin(e)) return out;
    const int64_t tiles = ((M + e.tile_m - 1) / e.tile_m) * ((N + e.tile_n - 1) / e.tile_n);
    const int64_t ksteps = (K + e.bk - 1) / e.bk;
    const int64_t ncu = std::max<int32_t>(m.cu_count, 1);
    for (int ks = 2; ks <= kMaxSplits && 2 * ks <= ksteps && tiles * (ks / 2) < 2 * ncu; ks *= 2) out.push_back(ks);
    return out;
}

double estimate_seconds(const pk_machine &m, const KernelEntry &e, int dtype, int64_t M, int64_t N, int64_t K,
                        bool wide, int ks) {
    // Per compute unit: the busiest one holds ceil(tiles / NCU) tiles, `res`
    // of them resident at once; each K step of a round costs the larger of
    // the resident tiles' arithmetic at the unit's rate and one step's
    // latency.  The rate falls when few wavefronts share a SIMD to hide LDS
    // and memory latency (full at about three per SIMD), and for MFMA tiles
    // with the LDS words each output needs (1/tile_m + 1/tile_n).
    const double clock = (m.clock_khz > 0 ? m.clock_khz : 2400000) * 1e3;
    const int64_t ncu = std::max<int32_t>(m.cu_count, 1);
    const int wave = m.wave > 0 ? m.wave : 64;
    const int64_t tm = (M + e.tile_m - 1) / e.tile_m, tn = (N + e.tile_n - 1) / e.tile_n;
    ks = std::max(ks, 1);
    // a product split along K runs ks workgroups per tile, each over its share
    const int64_t tiles = std::max<int64_t>(tm * tn, 1) * ks;
    const int64_t per_cu = (tiles + ncu - 1) / ncu;
    const int64_t res = std::min(blocks_per_cu(m, e), per_cu);
    const int64_t rounds = (per_cu + res - 1) / res;
    const int bk = e.bk > 0 ? e.bk : 1;
    const double ksteps = std::ceil((double)((std::max<int64_t>(K, 1) + bk - 1) / bk) / ks);
    const double flops_step = 2.0 * e.tile_m * e.tile_n * bk;
    const double waves_per_simd = (double)res * ((e.threads + wave - 1) / wave) / 4.0;
    const bool mfma = e.family == PK_FAMILY_MFMA;
    const bool vi32 = !mfma && dtype == PK_I32;  // int32 VALU: its own fitted barrier cost
    const double occupancy = std::min(1.0, std::pow(waves_per_simd / 3.0, mfma ? 0.4 : 0.25));
    // MFMA: the tile's LDS words per output; VALU: workgroups of fewer than
    // 256 work-items lose in proportion
    const double eff = mfma ? 0.85 / (1.0 + 6.0 * (1.0 / e.tile_m + 1.0 / e.tile_n))
                            : std::min(1.0, e.threads / 256.0);
    const double rate = cu_rate(m, e, dtype) * clock * eff * occupancy;
    const double latency = mfma ? ((e.variant & PK_MFMA_SINGLE) ? 0.4e-6 : 0.3e-6) : 0.1e-6;
    // VALU K steps also pay their two barriers per resident workgroup
    const double overhead = mfma ? 0.0 : (vi32 ? 0.1e-6 : 0.4e-6) * (double)res;
    // element loads instead of 16-byte loads (rows not aligned): measured
    // about 1.4x (f32) and 3.5x (bf16) slower per step, measured with the
    // same programs both ways at 2048^3 and 4096^3
    const double narrow = (mfma && !wide) ? (dtype == PK_BF16 ? 3.5 : dtype == PK_I32 ? 1.2 : 1.4) : 1.0;
    const double compute =
        narrow * (double)rounds * ksteps * (std::max((double)res * flops_step / rate, latency) + overhead);
    const double es = elem_bytes(dtype);
    // each workgroup reads its A and B panels over its share of K
    const double tile_bytes = es * (double)tiles * std::ceil((double)K / ks) * (e.tile_m + e.tile_n);
    const double hbm = (es * ((double)M * K + (double)K * N) + 4.0 * (double)M * N) / kHbmBytesPerSecond;
    // shares of K: clearing C (a second launch) and one atomic addition per
    // output and share
    const double split = ks > 1 ? kLaunchSeconds + 4.0 * (double)M * N / kHbmBytesPerSecond +
                                      (double)ks * M * N / kAtomicAddsPerSecond
                                : 0.0;
    return std::max(compute, std::max(tile_bytes / kHbmBytesPerSecond, hbm)) + split + kLaunchSeconds;
}

double tile_work_seconds(const pk_machine &m, const KernelEntry &e, int dtype, int64_t M, int64_t N, int64_t K) {
    // compute-unit seconds of the product's tiles when the unit is kept full
    // of this program's workgroups: a unit advances its resident tiles by one
    // K step in max(res * flops_step / rate, latency)
    const double clock = (m.clock_khz > 0 ? m.clock_khz : 2400000) * 1e3;
    const int wave = m.wave > 0 ? m.wave : 64;
    const int64_t tiles = ((M + e.tile_m - 1) / e.tile_m) * ((N + e.tile_n - 1) / e.tile_n);
    const int64_t res = blocks_per_cu(m, e);
    const int bk = e.bk > 0 ? e.bk : 1;
    const double ksteps = (double)((std::max<int64_t>(K, 1) + bk - 1) / bk);
    const double flops_step = 2.0 * e.tile_m * e.tile_n * bk;
    const double waves_per_simd = (double)res * ((e.threads + wave - 1) / wave) / 4.0;
    const double occupancy = std::min(1.0, std::pow(waves_per_simd / 3.0, 0.25));
    const bool mfma = e.family == PK_FAMILY_MFMA;
    const double eff = mfma ? 0.85 / (1.0 + 6.0 * (1.0 / e.tile_m + 1.0 / e.tile_n))
                            : std::min(1.0, e.threads / 256.0);
    const double rate = cu_rate(m, e, dtype) * clock * eff * occupancy;
    const double latency = mfma ? ((e.variant & PK_MFMA_SINGLE) ? 0.4e-6 : 0.3e-6) : 0.1e-6;
    const double step = std::max((double)res * flops_step / rate, latency);
    return (double)tiles * ksteps * step / (double)res;
}

void fill_params(const pk_table *tbl, const Candidate &c, int dtype, pk_params *out) {
    const pk_table::Part *part = tbl->part(c.family, dtype);
    point_params(c.family, part->fam.points[c.point], out);
    out->leaf = c.leaf;
    out->variant = c.variant;
    out->ks = c.ks > 1 ? c.ks : 0;
}

std::vector<Candidate> feasible(const pk_table *tbl, int dtype, int64_t M, int64_t N, int64_t K, const void *A,
                                int64_t lda, const void *B, int64_t ldb) {
    std::vector<Candidate> out;
    for (int family : {PK_FAMILY_VALU, PK_FAMILY_VALU2, PK_FAMILY_MFMA}) {  // the product families
        const pk_table::Part *part = tbl->part(family, dtype);
        if (!part || !part->supported) continue;
        // MFMA programs read unaligned rows element by element: feasible, slower
        const bool wide = !A || family != PK_FAMILY_MFMA || wide_rows(dtype, A, lda, B, ldb);
        for (size_t i = 0; i < part->fam.points.size(); ++i) {
            const int leaf = part->first_leaf[i];
            if (leaf < 0) continue;
            Candidate c;
            c.family = family;
            c.point = (int)i;
            c.leaf = leaf;
            c.variant = (int)part->solved.leaves[leaf].applied;
            c.entry = find_instance(family, c.variant, dtype, part->fam.points[i]);
            if (!c.entry || (!wide && !element_twin(*c.entry))) continue;
            c.estimate = estimate_seconds(tbl->machine, *c.entry, dtype, M, N, K, wide);
            out.push_back(c);
            for (int ks : k_splits(tbl->machine, *c.entry, M, N, K)) {  // the same program split along K
                Candidate d = c;
                d.ks = ks;
                d.estimate = estimate_seconds(tbl->machine, *c.entry, dtype, M, N, K, wide, ks);
                out.push_back(d);
            }
        }
    }
    return out;
}

// Times every candidate on the table's device.  Every HIP call is checked: a
// candidate whose launches or events fail is recorded as +inf (it can never
// be the pick), and a failure of the timing set-up itself is returned.
int time_candidates(const pk_table *tbl, int dtype, int64_t M, int64_t N, int64_t K,
                    const std::vector<Candidate> &cands, std::vector<double> *secs, const Operands *ops, int *best_out) {
    *best_out = -1;
    secs->assign(cands.size(), std::numeric_limits<double>::infinity());
    if (tbl->device < 0) return fail(PK_ERR_INVALID_ARG, "timing needs a table bound to a device");
    hipError_t err = hipSetDevice(tbl->device);
    if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(err));
    const size_t es = dtype == PK_BF16 ? 2 : 4;
    void *sA = nullptr, *sB = nullptr, *sC = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&]() {
        if (s) (void)hipStreamSynchronize(s);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
        if (sA) (void)hipFree(sA);
        if (sB) (void)hipFree(sB);
        if (sC) (void)hipFree(sC);
    };
    auto setup_failed = [&](const char *what, hipError_t e) {
        release();
        return fail(PK_ERR_HIP, std::string("timing set-up, ") + what + ": " + hipGetErrorString(e));
    };
    MmArgs args{nullptr, nullptr, nullptr, K, N, N, (int32_t)M, (int32_t)N, (int32_t)K, 0, 0};
    if (ops && ops->A) {
        args.A = ops->A;
        args.B = ops->B;
        args.C = ops->C;
        args.lda = ops->lda;
        args.ldb = ops->ldb;
        args.ldc = ops->ldc;
    } else {
        // scratch operands with a non-zero byte pattern (0x3c: about 0.0115 in
        // float32 and bfloat16), so the timed kernels do real arithmetic
        const size_t bA = std::max<size_t>(es * M * K, 16), bB = std::max<size_t>(es * K * N, 16),
                     bC = std::max<size_t>(4 * M * N, 16);
        if ((err = hipMalloc(&sA, bA)) != hipSuccess) return setup_failed("hipMalloc", err);
        if ((err = hipMalloc(&sB, bB)) != hipSuccess) return setup_failed("hipMalloc", err);
        if ((err = hipMalloc(&sC, bC)) != hipSuccess) return setup_failed("hipMalloc", err);
        if ((err = hipMemset(sA, 0x3c, bA)) != hipSuccess) return setup_failed("hipMemset", err);
        if ((err = hipMemset(sB, 0x3c, bB)) != hipSuccess) return setup_failed("hipMemset", err);
        args.A = sA;
        args.B = sB;
        args.C = sC;
    }
    args.vec = wide_rows(dtype, args.A, args.lda, args.B, args.ldb) ? 1 : 0;
    if ((err = hipStreamCreate(&s)) != hipSuccess) return setup_failed("hipStreamCreate", err);
    if ((err = hipEventCreate(&e0)) != hipSuccess) return setup_failed("hipEventCreate", err);
    if ((err = hipEventCreate(&e1)) != hipSuccess) return setup_failed("hipEventCreate", err);
    int best = -1;
    double best_t = std::numeric_limits<double>::infinity();
    // the most promising candidates first (least CASE estimate), so that the
    // best time so far is known early and slow candidates are cut short
    std::vector<size_t> order(cands.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return cands[x].estimate < cands[y].estimate; });
    for (size_t i : order) {
        const KernelEntry &e = *cands[i].entry;
        MmArgs ca = args;
        ca.splits = cands[i].ks > 1 ? cands[i].ks : 0;
        // warm-up launch, itself timed: a candidate whose one launch already
        // takes over a millisecond (launch latency is then negligible) and
        // twice the best mean so far cannot win; its one-launch time is kept
        float wms = 0.f;
        if (hipEventRecord(e0, s) != hipSuccess || launch(tbl->machine, e, ca, s) != PK_OK ||
            hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&wms, e0, e1) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipStreamSynchronize(s);
            continue;
        }
        if (wms > 1.f && wms * 1e-3 > 2.0 * best_t) {
            (*secs)[i] = wms * 1e-3;
            continue;
        }
        // back-to-back launches between two events, at least 3, up to about
        // 20 ms of work; after the first 3 a candidate already 1.5x slower
        // than the best so far cannot win and is not timed further (its mean
        // over those 3 is kept: a single launch between events would also
        // count the launch latency, which for small kernels exceeds the
        // kernel, and would cut off candidates that could win)
        float ms = 0.f;
        bool ok = hipEventRecord(e0, s) == hipSuccess;
        int reps = 0;
        while (ok) {
            ok = launch(tbl->machine, e, ca, s) == PK_OK;
            ++reps;
            if (ok && (reps == 3 || reps % 8 == 0)) {
                ok = hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
                if (ok && reps == 3 && ms * 1e-3 / 3 > 1.5 * best_t) break;
            }
            if (reps >= 3 && (ms >= 20.f || reps >= 200)) break;
        }
        if (!ok || !(ms > 0.f)) {
            (void)hipGetLastError();  // this candidate only: leave it at +inf
            (void)hipStreamSynchronize(s);
            continue;
        }
        const double t = ms * 1e-3 / reps;
        (*secs)[i] = t;
        if (t < best_t) {
            best_t = t;
            best = (int)i;
        }
    }
    err = hipStreamSynchronize(s);
    release();
    if (err != hipSuccess) return fail(PK_ERR_HIP, std::string("timing: ") + hipGetErrorString(err));
    if (best < 0) return fail(PK_ERR_HIP, "no candidate could be launched and timed");
    *best_out = best;
    return PK_OK;
}

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
    const pk_costmodel *model = (dtype >= 0 && dtype < 3) ? tbl->costmodel[dtype].get() : nullptr;
    if (policy == PK_POLICY_LEARNED && model) {
        // order by predicted time; near-ties are settled by measurement
        std::vector<float> X(cands.size() * PK_NFEATURES), pred(cands.size());
        const bool wide = !A || wide_rows(dtype, A, lda, B, ldb);
        for (size_t i = 0; i < cands.size(); ++i)
            features(tbl->machine, *cands[i].entry, dtype, M, N, K, wide, cands[i].ks, &X[i * PK_NFEATURES]);
        costmodel_predict(*model, tbl->device, X.data(), (int64_t)cands.size(), pred.data());
        std::vector<int> order(cands.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return pred[a] < pred[b]; });
        pick = order[0];
        tbl->learned_selections++;
        // candidates predicted within the table's margin of the best (5 % by
        // default) are too close for the model to order: they are measured
        const double margin = tbl->learned_margin;
        if (margin > 0.0 && order.size() > 1 && std::exp((double)pred[order[1]] - pred[order[0]]) < 1.0 + margin) {
            std::vector<Candidate> close;
            std::vector<int> idx;
            for (int i : order)
                if (std::exp((double)pred[i] - pred[order[0]]) <= 1.0 + margin) {
                    close.push_back(cands[i]);
                    idx.push_back(i);
                }
            std::vector<double> secs;
            Operands ops{A, lda, B, ldb, nullptr, 0};
            void *C = nullptr;
            if (A) {
                if (hipMalloc(&C, std::max<size_t>(4 * M * N, 16)) != hipSuccess)
                    return fail(PK_ERR_HIP, "learned selection: allocation failed");
                ops.C = C;
                ops.ldc = N;
            }
            int f = -1;
            const int rc = time_candidates(tbl, dtype, M, N, K, close, &secs, A ? &ops : nullptr, &f);
            if (C) (void)hipFree(C);
            if (rc != PK_OK) return rc;
            pick = idx[f];
            tbl->learned_fallbacks++;
            tbl->learned_measured += (int64_t)close.size();
        }
        fill_params(tbl, cands[pick], dtype, out);
    } else if (policy == PK_POLICY_CASE || policy == PK_POLICY_LEARNED) {
        for (size_t i = 1; i < cands.size(); ++i)
            if (cands[i].estimate < cands[pick].estimate) pick = (int)i;
        fill_params(tbl, cands[pick], dtype, out);
        if (policy == PK_POLICY_LEARNED)
            return fail(PK_ERR_COST_MODEL, "no cost model for this dtype loaded; CASE pick returned");
    } else if (policy == PK_POLICY_EXHAUSTIVE) {
        std::vector<double> secs;
        Operands ops{A, lda, B, ldb, nullptr, 0};
        void *C = nullptr;
        if (A) {  // time on the caller's data needs an output: scratch C
            if (hipMalloc(&C, std::max<size_t>(4 * M * N, 16)) != hipSuccess)
                return fail(PK_ERR_HIP, "exhaustive selection: allocation failed");
            ops.C = C;
            ops.ldc = N;
        }
        const int rc = time_candidates(tbl, dtype, M, N, K, cands, &secs, A ? &ops : nullptr, &pick);
        if (C) (void)hipFree(C);
        if (rc != PK_OK) return rc;
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
