// Matrix-core (MFMA) kernels of the matrix product for gfx950.
//
// Same contract as the VALU family (C = [C +] A B, row-major, any M, N, K),
// used where the product is a dense contraction in float32 or bfloat16:
//   float32:  v_mfma_f32_32x32x2_f32   (A 32x2, B 2x32, C 32x32 per wavefront)
//   bfloat16: v_mfma_f32_32x32x16_bf16 (A 32x16, B 16x32, float32 accumulate)
//
// Decomposition: a workgroup of WM x WN wavefronts owns a BM x BN output tile;
// each wavefront owns (BM/WM) x (BN/WN), i.e. TM x TN blocks of 32x32
// accumulators (16 per lane each).  K advances in steps of BK through LDS:
//   float32:  As[BM][BK+4]   (k contiguous),   Bs[BK][BN+4]   (n contiguous)
//   bfloat16: As[BM][BK+8]   (k contiguous),   Bs[BK][BN+32]  (n contiguous;
//             each lane gathers its 8 k values of a column with two of
//             gfx950's transposing LDS reads)
// STAGES = 2 double-buffers the tiles (one barrier per K step: the next tile is
// fetched from global memory into registers while the current one is
// consumed); STAGES = 1 keeps one buffer and two barriers per step, as in the
// paper's kernel, with the next step's loads in flight in registers while the
// current step multiplies out of LDS.  LDS bytes = STAGES * (A tile + B tile).
// Left to itself, the compiler's scheduler sinks those loads to the end of the
// step (shortening their registers' lives) and the step then waits out a whole
// global-memory latency; a scheduling barrier keeps them ahead of the products
// in programs whose wavefronts hold at least a 64 x 64 tile (few wavefronts per
// SIMD to hide the latency otherwise) and in every single-stage program.
//
// The order in which k enters each 32x32 block's sum is permuted: lanes 0-31
// consume k in the first half of the LDS tile and lanes 32-63 the second half,
// so a lane's operands are contiguous in LDS.  The set of products summed is
// unchanged.
//
// Global loads are 16 bytes wide, so the leading dimensions must keep rows
// aligned (lda, ldb multiples of 4 floats / 8 bfloat16 and 16-byte aligned
// bases); the host checks this and otherwise launches the element-load twin.
// Tiles crossing the matrix edge
// keep the wide loads: they clamp the rows of A and the column chunks of B
// they read to the last chunk in range (results outside C are never stored),
// zero the elements of A at k >= K, read the rows of B at k >= K from a block
// of zeros, and guard their stores.  Edge loads choose an address, never a
// loaded value, so they carry no branches and stay in flight together.
//
// Workgroup -> tile map: workgroups are dispatched round-robin over the 8 XCDs
// (each with its own L2); blocks b and b+8 land on the same XCD, so the map
// first gives each XCD a contiguous range of tile indices and then walks that
// range in groups of GROUP_M tile rows, which keeps the A and B panels an XCD
// reads within its L2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kargs.hpp"

namespace pkk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Pointers into global memory.  The grouped kernels read operand pointers
// from descriptors in memory, where the compiler cannot infer the address
// space and would emit flat accesses (which also wait on the LDS counter).
template <class T> using gptr = const __attribute__((address_space(1))) T *;
template <class T> using gmut = __attribute__((address_space(1))) T *;

// the source of every element at k >= K (read only)
static __device__ __attribute__((aligned(16))) unsigned int kZeroBlock[4] = {0u, 0u, 0u, 0u};

constexpr int XCDS = kXcds;
constexpr int GROUP_M = 8;

// tile (tm, tn) of linear workgroup b among tiles_m x tiles_n
__device__ __forceinline__ void tile_of(int64_t b, int tiles_m, int tiles_n, int *tm, int *tn) {
    const int64_t T = (int64_t)tiles_m * tiles_n;
    const int64_t q = T / XCDS;
    int64_t pid = b;
    if (b < q * XCDS) pid = (b % XCDS) * q + b / XCDS;
    const int64_t width = (int64_t)GROUP_M * tiles_n;
    const int64_t group = pid / width;
    const int first_m = (int)(group * GROUP_M);
    const int gm = min(tiles_m - first_m, GROUP_M);
    const int64_t in = pid % width;
    *tm = first_m + (int)(in % gm);
    *tn = (int)(in / gm);
}

// ------------------------------------------------------------------ float32
// LDS floats of a float32 tile program: STAGES x (A tile BM x (BK + 4)),
// then STAGES x (B tile BK x (BN + 4)); every part starts 16-byte aligned.
template <int BM, int BN, int BK, int STAGES> struct F32Lds {
    static constexpr int LDA_S = BK + 4, LDB_S = BN + 4;
    static constexpr int A = BM * LDA_S, B = BK * LDB_S;
    static constexpr int floats = STAGES * (A + B);
};

// One BM x BN output tile at (row0, col0) over the K steps [kt0, kt1) (of
// BK each), its A tiles at As0 (STAGES x F32Lds::A floats) and its B tiles
// at Bs0 (STAGES x F32Lds::B floats) in LDS.  `vec`: the rows
// of A and B are 16-byte aligned, so interior tiles may use 16-byte loads.
// With a.splits > 1 the tile's sum over its K steps is added to C atomically
// (C holds zeros or the sums of the other shares of K); otherwise it is
// stored (added to C with a.accumulate).  The caller synchronises the
// workgroup before reusing the LDS for another tile.

template <int BM, int BN, int BK, int WM, int WN, int STAGES, bool EDGE_ADDR>
__device__ __forceinline__ void mfma_f32_tile(const MmArgs &a, const int row0, const int col0, const bool vec,
                                              float *const As0, float *const Bs0, const int kt0,
                                              const int kt1) {
    constexpr int NT = 64 * WM * WN;
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 32, TN = WTN / 32;
    using L = F32Lds<BM, BN, BK, STAGES>;
    constexpr int LDA_S = L::LDA_S, LDB_S = L::LDB_S;
    constexpr int A4 = BM * BK / 4 / NT;  // float4 loads per work-item per A tile
    constexpr int B4 = BK * BN / 4 / NT;
    static_assert(TM >= 1 && TN >= 1 && WTM % 32 == 0 && WTN % 32 == 0, "wave tile must be 32x32 blocks");
    static_assert(A4 >= 1 && B4 >= 1 && (BM * BK / 4) % NT == 0 && (BK * BN / 4) % NT == 0, "tile loads");
    static_assert(BK % 8 == 0, "BK");
    constexpr bool PIN = TM * TN >= 4;  // two stages: the next step's loads ahead of the products


    // the operands from this workgroup's first K step on: its steps run from
    // 0, and K counts what is left of the product from there (the same loops
    // and guards serve a whole product and a share of one)
    const gptr<float> __restrict__ A = (gptr<float>)a.A + kt0 * BK;
    const gptr<float> __restrict__ B = (gptr<float>)a.B + (int64_t)kt0 * BK * a.ldb;
    const gmut<float> __restrict__ C = (gmut<float>)a.C;
    const int M = a.M, N = a.N, K = a.K - kt0 * BK;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int r = lane & 31, h = lane >> 5;

    const bool interior = (row0 + BM <= M) && (col0 + BN <= N);
    // a wavefront whose part of an edge tile lies wholly outside C has nothing
    // to multiply (it still loads and stores its share of the operand tiles);
    // skipping its products frees the matrix unit for the other wavefronts
    // (not in programs of 1024 work-items, whose registers are at the limit)
    const bool idle = NT <= 512 && ((row0 + wm * WTM >= M) || (col0 + wn * WTN >= N));

    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

    f32x4 ra[A4], rb[B4];
    // a K step that lies wholly inside aligned operands: no guards, so the
    // loads issue back to back (guarded loads branch per load, and the
    // compiler then waits for each load before the next)
    auto gload_fast = [&](int k0) {
#pragma unroll
        for (int u = 0; u < A4; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BK / 4), c4 = (f % (BK / 4)) * 4;
            ra[u] = *reinterpret_cast<gptr<f32x4>>(A + (int64_t)(row0 + rr) * a.lda + k0 + c4);
        }
#pragma unroll
        for (int u = 0; u < B4; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BN / 4), c4 = (f % (BN / 4)) * 4;
            rb[u] = *reinterpret_cast<gptr<f32x4>>(B + (int64_t)(k0 + rr) * a.ldb + col0 + c4);
        }
    };
    // Any K step, edge tiles included.  Without EDGE_ADDR: guarded loads
    // (16 bytes where the chunk is wholly inside the matrix, else element by
    // element), which hold fewer registers where edge steps are rare.
    // EDGE_ADDR, for programs whose steps are mostly edge steps (many small
    // products): every load goes to a chosen address.  Aligned rows (vec):
    // 16-byte loads at addresses clamped into the matrix.
    // Rows of A past M read row M - 1 and columns of B past N read the chunk
    // holding column N - 1 (their results are never stored); in a step past
    // the end of K, A's chunks past k = K - 1 read the chunk holding it and
    // the elements at k >= K become zeros, and the rows of B at k >= K read a
    // block of zeros.  Every chunk read holds an element of the matrix, so it
    // lies inside its aligned row.
    // Unaligned rows: element loads.
    auto gload = [&](int k0) {
        if constexpr (!EDGE_ADDR) {
            const bool kfull = (k0 + BK <= K);
#pragma unroll
            for (int u = 0; u < A4; ++u) {
                const int f = tid + u * NT;
                const int rr = f / (BK / 4), c4 = (f % (BK / 4)) * 4;
                const int gr = row0 + rr, gc = k0 + c4;
                if (vec && kfull && gr < M) {
                    ra[u] = *reinterpret_cast<gptr<f32x4>>(A + (int64_t)gr * a.lda + gc);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        ra[u][e] = (gr < M && gc + e < K) ? A[(int64_t)gr * a.lda + gc + e] : 0.0f;
                }
            }
#pragma unroll
            for (int u = 0; u < B4; ++u) {
                const int f = tid + u * NT;
                const int rr = f / (BN / 4), c4 = (f % (BN / 4)) * 4;
                const int gr = k0 + rr, gc = col0 + c4;
                if (vec && gr < K && gc + 4 <= N) {
                    rb[u] = *reinterpret_cast<gptr<f32x4>>(B + (int64_t)gr * a.ldb + gc);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        rb[u][e] = (gr < K && gc + e < N) ? B[(int64_t)gr * a.ldb + gc + e] : 0.0f;
                }
            }
            return;
        }
        const gptr<float> zero = (gptr<float>)(const void *)kZeroBlock;
        if (vec) {
            const int klast = (K - 1) & ~3, nlast = (N - 1) & ~3;
            if (k0 + BK <= K) {
#pragma unroll
                for (int u = 0; u < A4; ++u) {
                    const int f = tid + u * NT;
                    const int rr = f / (BK / 4), c4 = (f % (BK / 4)) * 4;
                    ra[u] = *reinterpret_cast<gptr<f32x4>>(A + (int64_t)min(row0 + rr, M - 1) * a.lda + k0 + c4);
                }
            } else {
#pragma unroll
                for (int u = 0; u < A4; ++u) {
                    const int f = tid + u * NT;
                    const int rr = f / (BK / 4), c4 = (f % (BK / 4)) * 4;
                    const int k = k0 + c4;
                    f32x4 v = *reinterpret_cast<gptr<f32x4>>(A + (int64_t)min(row0 + rr, M - 1) * a.lda +
                                                             min(k, klast));
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] = k + e < K ? v[e] : 0.0f;
                    ra[u] = v;
                }
            }
#pragma unroll
            for (int u = 0; u < B4; ++u) {
                const int f = tid + u * NT;
                const int rr = f / (BN / 4), c4 = (f % (BN / 4)) * 4;
                const int k = k0 + rr;
                rb[u] = *reinterpret_cast<gptr<f32x4>>(k < K ? B + (int64_t)k * a.ldb + min(col0 + c4, nlast) : zero);
            }
            return;
        }
#pragma unroll
        for (int u = 0; u < A4; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BK / 4), c4 = (f % (BK / 4)) * 4;
            const gptr<float> row = A + (int64_t)min(row0 + rr, M - 1) * a.lda;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = k0 + c4 + e;
                ra[u][e] = *(k < K ? row + k : zero);
            }
        }
#pragma unroll
        for (int u = 0; u < B4; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BN / 4), c4 = (f % (BN / 4)) * 4;
            const int k = k0 + rr;
            const gptr<float> row = k < K ? B + (int64_t)k * a.ldb : nullptr;
#pragma unroll
            for (int e = 0; e < 4; ++e) rb[u][e] = *(row ? row + min(col0 + c4 + e, N - 1) : zero);
        }
    };
    auto sstore = [&](int st) {
#pragma unroll
        for (int u = 0; u < A4; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BK / 4), c4 = (f % (BK / 4)) * 4;
            *reinterpret_cast<f32x4 *>(&As0[st * L::A + rr * LDA_S + c4]) = ra[u];
        }
#pragma unroll
        for (int u = 0; u < B4; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BN / 4), c4 = (f % (BN / 4)) * 4;
            *reinterpret_cast<f32x4 *>(&Bs0[st * L::B + rr * LDB_S + c4]) = rb[u];
        }
    };
    auto compute = [&](int st) {
        const float *as = &As0[st * L::A + (wm * WTM + r) * LDA_S + h * (BK / 2)];
        const float *bs = &Bs0[st * L::B + (h * (BK / 2)) * LDB_S + wn * WTN + r];
#pragma unroll
        for (int kc = 0; kc < BK / 2; kc += 4) {
            f32x4 af[TM];
            float bf[TN][4];
#pragma unroll
            for (int i = 0; i < TM; ++i) af[i] = *reinterpret_cast<const f32x4 *>(as + i * 32 * LDA_S + kc);
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) bf[j][q] = bs[(kc + q) * LDB_S + j * 32];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int i = 0; i < TM; ++i)
#pragma unroll
                    for (int j = 0; j < TN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][q], bf[j][q], acc[i][j], 0, 0, 0);
        }
    };

    // the workgroup's KT K steps (all of K, or its share of a product split
    // along K).  Leading steps that need no guards: all of them for an
    // interior tile on aligned rows, except a partial last one.
    const int KT = kt1 - kt0;
    const int KF = (vec && interior) ? min(K / BK, KT) : 0;
    if (STAGES == 2) {
        if (KT > 0) {
            if (KF > 0)
                gload_fast(0);
            else
                gload(0);
            sstore(0);
        }
        __syncthreads();
        int kt = 0;
        // steps whose successor is unguarded too: a loop without branches, so
        // the next step's loads stay in flight while this step multiplies
        for (; kt + 1 < KF; ++kt) {
            const int cur = kt & 1;
            gload_fast((kt + 1) * BK);
            if constexpr (PIN) __builtin_amdgcn_sched_barrier(0);
            compute(cur);
            sstore(cur ^ 1);
            __syncthreads();
        }
        for (; kt < KT; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < KT) gload((kt + 1) * BK);
            if constexpr (PIN) __builtin_amdgcn_sched_barrier(0);
            if (!idle) compute(cur);
            if (kt + 1 < KT) sstore(cur ^ 1);
            __syncthreads();
        }
    } else {
        // one LDS buffer: step kt + 1's loads are in flight (in registers)
        // while step kt multiplies out of LDS
        if (KT > 0) {
            if (KF > 0)
                gload_fast(0);
            else
                gload(0);
        }
        int kt = 0;
        for (; kt + 1 < KF; ++kt) {
            __syncthreads();  // the previous step's LDS reads are done
            sstore(0);
            __syncthreads();
            gload_fast((kt + 1) * BK);
            __builtin_amdgcn_sched_barrier(0);
            compute(0);
        }
        for (; kt < KT; ++kt) {
            __syncthreads();
            sstore(0);
            __syncthreads();
            if (kt + 1 < KT) gload((kt + 1) * BK);
            __builtin_amdgcn_sched_barrier(0);
            if (!idle) compute(0);
        }
    }

    // epilogue: value v of block (i, j) is row 8*(v/4) + 4*h + v%4, column r
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int gc = col0 + wn * WTN + j * 32 + r;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int gr = row0 + wm * WTM + i * 32 + 8 * (v / 4) + 4 * h + (v % 4);
                if (interior || (gr < M && gc < N)) {
                    const gmut<float> p = C + (int64_t)gr * a.ldc + gc;
                    if (a.splits > 1)  // a share of K: added to C, which holds the other shares' sums
                        unsafeAtomicAdd((float *)p, acc[i][j][v]);
                    else
                        *p = a.accumulate ? *p + acc[i][j][v] : acc[i][j][v];
                }
            }
        }
}

// ------------------------------------------------------------------ bfloat16
// LDS elements (16-bit) of a bfloat16 tile program: STAGES x (A tile BM x
// (BK + 8)), then STAGES x (B tile BK x (BN + 32), row-major as in memory).
// A B row spans BN + 32 elements, 64 bytes past a multiple of 256 for every BN
// here: the four rows one transposing read touches fall in four different
// 64-byte quarters of the banks.
template <int BM, int BN, int BK, int STAGES> struct Bf16Lds {
    static constexpr int LD_S = BK + 8, LDB_S = BN + 32;
    static constexpr int A = BM * LD_S, B = BK * LDB_S;
    static constexpr int elems = STAGES * (A + B);
};

// The MFMA B operand of lanes [16g, 16g + 16) from a row-major tile in LDS:
// gfx950's transposing read hands lane i of each group of 16 element i % 4 of
// the 8 bytes addressed by lane 4j + i / 4, for j = 0..3.  With lane m of the
// group addressing row m / 4, columns 4 (m % 4) .. + 3, lane i receives
// column i of four consecutive rows.
typedef short s16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ s16x4 lds_read_tr16(const unsigned short *p) {
    return __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) s16x4 *)p);
}

// bfloat16 tile, its A tiles at As0 (STAGES x Bf16Lds::A elements) and its B
// tiles at Bs0 (STAGES x Bf16Lds::B); `vec`: A and B rows 16-byte aligned.
template <int BM, int BN, int BK, int WM, int WN, int STAGES, bool EDGE_ADDR>
__device__ __forceinline__ void mfma_bf16_tile(const MmArgs &a, const int row0, const int col0, const bool vec,
                                               unsigned short *const As0, unsigned short *const Bs0,
                                               const int kt0, const int kt1) {
    constexpr int NT = 64 * WM * WN;
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 32, TN = WTN / 32;
    using L = Bf16Lds<BM, BN, BK, STAGES>;
    constexpr int LD_S = L::LD_S;                // row stride (elements) of the A tiles
    constexpr int LDB_S = L::LDB_S;              // row stride of the B tiles
    constexpr int A8 = BM * BK / 8 / NT;         // 16-byte loads per work-item per A tile
    constexpr int B8 = BK * BN / 8 / NT;         // 16-byte loads per work-item per B tile
    static_assert(TM >= 1 && TN >= 1 && WTM % 32 == 0 && WTN % 32 == 0, "wave tile must be 32x32 blocks");
    static_assert(A8 >= 1 && B8 >= 1 && (BM * BK / 8) % NT == 0 && (BK * BN / 8) % NT == 0, "tile loads");
    static_assert(BK % 32 == 0 && BN % 8 == 0, "BK, BN");
    static_assert((LDB_S * 2) % 256 == 64 || (LDB_S * 2) % 256 == 192, "B rows one quarter of the banks apart");
    constexpr bool PIN = true;  // two stages: the next step's loads ahead of the products

    // from this workgroup's first K step on, as in the float32 tile
    const gptr<unsigned short> __restrict__ A = (gptr<unsigned short>)a.A + kt0 * BK;
    const gptr<unsigned short> __restrict__ B = (gptr<unsigned short>)a.B + (int64_t)kt0 * BK * a.ldb;
    const gmut<float> __restrict__ C = (gmut<float>)a.C;
    const int M = a.M, N = a.N, K = a.K - kt0 * BK;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int r = lane & 31, h = lane >> 5;

    const bool interior = (row0 + BM <= M) && (col0 + BN <= N);
    // a wavefront whose part of an edge tile lies wholly outside C has nothing
    // to multiply (it still loads and stores its share of the operand tiles);
    // skipping its products frees the matrix unit for the other wavefronts
    // (not in programs of 1024 work-items, whose registers are at the limit)
    const bool idle = NT <= 512 && ((row0 + wm * WTM >= M) || (col0 + wn * WTN >= N));

    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

    // work-item f of the workgroup's u-th load: A row f / (BK / 8), its k
    // chunk (f % (BK / 8)) * 8; B row (k) f / (BN / 8), its column chunk
    // (f % (BN / 8)) * 8
    u16x8 ra[A8], rb[B8];
    auto gload_fast = [&](int k0) {  // unguarded, as in the float32 tile
#pragma unroll
        for (int u = 0; u < A8; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BK / 8), c8 = (f % (BK / 8)) * 8;
            ra[u] = *reinterpret_cast<gptr<u16x8>>(A + (int64_t)(row0 + rr) * a.lda + k0 + c8);
        }
#pragma unroll
        for (int u = 0; u < B8; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BN / 8), c8 = (f % (BN / 8)) * 8;
            rb[u] = *reinterpret_cast<gptr<u16x8>>(B + (int64_t)(k0 + rr) * a.ldb + col0 + c8);
        }
    };
    auto gload = [&](int k0) {  // any K step: as in the float32 tile
        if constexpr (!EDGE_ADDR) {
            const bool kfull = (k0 + BK <= K);
#pragma unroll
            for (int u = 0; u < A8; ++u) {
                const int f = tid + u * NT;
                const int rr = f / (BK / 8), c8 = (f % (BK / 8)) * 8;
                const int gr = row0 + rr, gc = k0 + c8;
                if (vec && kfull && gr < M) {
                    ra[u] = *reinterpret_cast<gptr<u16x8>>(A + (int64_t)gr * a.lda + gc);
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        ra[u][e] = (gr < M && gc + e < K) ? A[(int64_t)gr * a.lda + gc + e] : (unsigned short)0;
                }
            }
#pragma unroll
            for (int u = 0; u < B8; ++u) {
                const int f = tid + u * NT;
                const int rr = f / (BN / 8), c8 = (f % (BN / 8)) * 8;
                const int gr = k0 + rr, gc = col0 + c8;
                if (vec && gr < K && gc + 8 <= N) {
                    rb[u] = *reinterpret_cast<gptr<u16x8>>(B + (int64_t)gr * a.ldb + gc);
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        rb[u][e] = (gr < K && gc + e < N) ? B[(int64_t)gr * a.ldb + gc + e] : (unsigned short)0;
                }
            }
            return;
        }
        const gptr<unsigned short> zero = (gptr<unsigned short>)(const void *)kZeroBlock;
        if (vec) {
            // aligned rows: 16-byte chunks at chosen addresses.  A rows past M
            // repeat row M - 1 and B chunks past N the row's last chunk (their
            // products land outside C); B rows past K read the zero block; the
            // chunk holding A's k tail is masked
            const int klast = (K - 1) & ~7, nlast = (N - 1) & ~7;
            if (k0 + BK <= K) {
#pragma unroll
                for (int u = 0; u < A8; ++u) {
                    const int f = tid + u * NT;
                    const int rr = f / (BK / 8), c8 = (f % (BK / 8)) * 8;
                    ra[u] = *reinterpret_cast<gptr<u16x8>>(A + (int64_t)min(row0 + rr, M - 1) * a.lda + k0 + c8);
                }
            } else {
#pragma unroll
                for (int u = 0; u < A8; ++u) {
                    const int f = tid + u * NT;
                    const int rr = f / (BK / 8), c8 = (f % (BK / 8)) * 8;
                    const int k = k0 + c8;
                    u32x4 v = *reinterpret_cast<gptr<u32x4>>(A + (int64_t)min(row0 + rr, M - 1) * a.lda +
                                                             min(k, klast));
                    // word w holds k + 2w (low half) and k + 2w + 1 (high half)
#pragma unroll
                    for (int w = 0; w < 4; ++w)
                        v[w] &= k + 2 * w + 1 < K ? 0xffffffffu : (k + 2 * w < K ? 0x0000ffffu : 0u);
                    ra[u] = __builtin_bit_cast(u16x8, v);
                }
            }
#pragma unroll
            for (int u = 0; u < B8; ++u) {
                const int f = tid + u * NT;
                const int rr = f / (BN / 8), c8 = (f % (BN / 8)) * 8;
                const int k = k0 + rr;
                rb[u] = *(k < K ? reinterpret_cast<gptr<u16x8>>(B + (int64_t)k * a.ldb + min(col0 + c8, nlast))
                                : (gptr<u16x8>)(const void *)kZeroBlock);
            }
            return;
        }
#pragma unroll
        for (int u = 0; u < A8; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BK / 8), c8 = (f % (BK / 8)) * 8;
            const gptr<unsigned short> row = A + (int64_t)min(row0 + rr, M - 1) * a.lda;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + c8 + e;
                ra[u][e] = *(k < K ? row + k : zero);
            }
        }
#pragma unroll
        for (int u = 0; u < B8; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BN / 8), c8 = (f % (BN / 8)) * 8;
            const int k = k0 + rr;
            const gptr<unsigned short> row = k < K ? B + (int64_t)k * a.ldb : nullptr;
#pragma unroll
            for (int e = 0; e < 8; ++e) rb[u][e] = *(row ? row + min(col0 + c8 + e, N - 1) : zero);
        }
    };
    auto sstore = [&](int st) {
#pragma unroll
        for (int u = 0; u < A8; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BK / 8), c8 = (f % (BK / 8)) * 8;
            *reinterpret_cast<u16x8 *>(&As0[st * L::A + rr * LD_S + c8]) = ra[u];
        }
#pragma unroll
        for (int u = 0; u < B8; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BN / 8), c8 = (f % (BN / 8)) * 8;
            *reinterpret_cast<u16x8 *>(&Bs0[st * L::B + rr * LDB_S + c8]) = rb[u];
        }
    };
    // lane (r, h) multiplies A row r and B column r over k = h BK/2 + kc + t,
    // t = 0..7, per MFMA; its B values come from two transposing reads (t =
    // 0..3, then 4..7): lane m of its group of 16 addresses row m / 4 of the
    // four, columns 4 (m % 4) .. + 3 of the group's 16 (groups 0 and 2 take
    // columns 0..15 of the block, 1 and 3 columns 16..31)
    const int grp = lane >> 4, m16 = lane & 15;
    auto compute = [&](int st) {
        const unsigned short *as = &As0[st * L::A + (wm * WTM + r) * LD_S + h * (BK / 2)];
        const unsigned short *bs = &Bs0[st * L::B + (h * (BK / 2) + (m16 >> 2)) * LDB_S + wn * WTN +
                                        16 * (grp & 1) + 4 * (m16 & 3)];
#pragma unroll
        for (int kc = 0; kc < BK / 2; kc += 8) {
            bf16x8 af[TM], bf[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) af[i] = *reinterpret_cast<const bf16x8 *>(as + i * 32 * LD_S + kc);
#pragma unroll
            for (int j = 0; j < TN; ++j) {
                const s16x4 lo = lds_read_tr16(bs + kc * LDB_S + j * 32);
                const s16x4 hi = lds_read_tr16(bs + (kc + 4) * LDB_S + j * 32);
                bf[j] = __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
    };

    // the workgroup's KT K steps (all of K, or its share of a product split
    // along K).  Leading steps that need no guards: all of them for an
    // interior tile on aligned rows, except a partial last one.
    const int KT = kt1 - kt0;
    const int KF = (vec && interior) ? min(K / BK, KT) : 0;
    if (STAGES == 2) {
        if (KT > 0) {
            if (KF > 0)
                gload_fast(0);
            else
                gload(0);
            sstore(0);
        }
        __syncthreads();
        int kt = 0;
        // steps whose successor is unguarded too: a loop without branches, so
        // the next step's loads stay in flight while this step multiplies
        for (; kt + 1 < KF; ++kt) {
            const int cur = kt & 1;
            gload_fast((kt + 1) * BK);
            if constexpr (PIN) __builtin_amdgcn_sched_barrier(0);
            compute(cur);
            sstore(cur ^ 1);
            __syncthreads();
        }
        for (; kt < KT; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < KT) gload((kt + 1) * BK);
            if constexpr (PIN) __builtin_amdgcn_sched_barrier(0);
            if (!idle) compute(cur);
            if (kt + 1 < KT) sstore(cur ^ 1);
            __syncthreads();
        }
    } else {
        // one LDS buffer: step kt + 1's loads are in flight (in registers)
        // while step kt multiplies out of LDS
        if (KT > 0) {
            if (KF > 0)
                gload_fast(0);
            else
                gload(0);
        }
        int kt = 0;
        for (; kt + 1 < KF; ++kt) {
            __syncthreads();  // the previous step's LDS reads are done
            sstore(0);
            __syncthreads();
            gload_fast((kt + 1) * BK);
            __builtin_amdgcn_sched_barrier(0);
            compute(0);
        }
        for (; kt < KT; ++kt) {
            __syncthreads();
            sstore(0);
            __syncthreads();
            if (kt + 1 < KT) gload((kt + 1) * BK);
            __builtin_amdgcn_sched_barrier(0);
            if (!idle) compute(0);
        }
    }

#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int gc = col0 + wn * WTN + j * 32 + r;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int gr = row0 + wm * WTM + i * 32 + 8 * (v / 4) + 4 * h + (v % 4);
                if (interior || (gr < M && gc < N)) {
                    const gmut<float> p = C + (int64_t)gr * a.ldc + gc;
                    if (a.splits > 1)  // a share of K: added to C, which holds the other shares' sums
                        unsafeAtomicAdd((float *)p, acc[i][j][v]);
                    else
                        *p = a.accumulate ? *p + acc[i][j][v] : acc[i][j][v];
                }
            }
        }
}

// ------------------------------------------------------------------ single product
// Split along K (a.splits = S > 1): the grid holds S x tiles workgroups, share
// by share; workgroup b takes share b / tiles of tile b % tiles, the K steps
// [KT s / S, KT (s + 1) / S) of the product's KT = ceil(K / BK).  Programs of
// 1024 work-items are never split (kSplittableThreads): their registers are
// at the limit already.
template <int BK>
__device__ __forceinline__ void k_share(const MmArgs &a, int64_t tiles, int64_t *b, int *kt0, int *kt1) {
    const int KT = (a.K + BK - 1) / BK;
    *kt0 = 0;
    *kt1 = KT;
    if (a.splits > 1) {
        const int s = (int)(*b / tiles);
        *b -= (int64_t)s * tiles;
        *kt0 = (int)((int64_t)KT * s / a.splits);
        *kt1 = (int)((int64_t)KT * (s + 1) / a.splits);
    }
}

// WIDE: 16-byte loads along aligned rows; the element-load twin (WIDE =
// false) is a kernel of its own, so neither carries the other's load path.
// The twins of workgroups up to 256 work-items load at chosen addresses (all
// their steps take the edge path).  SPLIT: the kernel runs shares of K
// (a.splits > 1); the wide program's split form is a kernel of its own too,
// so the whole-product kernel carries none of it (the element-load twins,
// already off the fast path, split in place).
template <int BM, int BN, int BK, int WM, int WN, int STAGES, bool WIDE = true, bool SPLIT = !WIDE>
__device__ __forceinline__ void mfma_f32(const MmArgs &a0) {
    MmArgs a = a0;
    if constexpr (!SPLIT || 64 * WM * WN > kSplittableThreads) a.splits = 0;
    int tm, tn;
    using L = F32Lds<BM, BN, BK, STAGES>;
    __shared__ __attribute__((aligned(16))) float As[STAGES * L::A];
    __shared__ __attribute__((aligned(16))) float Bs[STAGES * L::B];
    int64_t b = blockIdx.x;
    int kt0, kt1;
    k_share<BK>(a, (int64_t)((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN), &b, &kt0, &kt1);
    tile_of(b, (a.M + BM - 1) / BM, (a.N + BN - 1) / BN, &tm, &tn);
    mfma_f32_tile<BM, BN, BK, WM, WN, STAGES, !WIDE && WM * WN < 8>(a, tm * BM, tn * BN, WIDE, As, Bs, kt0, kt1);
}

template <int BM, int BN, int BK, int WM, int WN, int STAGES, bool WIDE = true, bool SPLIT = !WIDE>
__device__ __forceinline__ void mfma_bf16(const MmArgs &a0) {
    MmArgs a = a0;
    if constexpr (!SPLIT || 64 * WM * WN > kSplittableThreads) a.splits = 0;
    int tm, tn;
    using L = Bf16Lds<BM, BN, BK, STAGES>;
    __shared__ __attribute__((aligned(16))) unsigned short As[STAGES * L::A];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[STAGES * L::B];
    int64_t b = blockIdx.x;
    int kt0, kt1;
    k_share<BK>(a, (int64_t)((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN), &b, &kt0, &kt1);
    tile_of(b, (a.M + BM - 1) / BM, (a.N + BN - 1) / BN, &tm, &tn);
    mfma_bf16_tile<BM, BN, BK, WM, WN, STAGES, !WIDE && WM * WN < 8>(a, tm * BM, tn * BN, WIDE, As, Bs, kt0, kt1);
}

// ------------------------------------------------------------------ grouped (persistent)
// Many independent products in one launch; tile t belongs to group
// tile_group[t] and is tile t - tile_start of that group, numbered row-major
// over its tiles (a product's tiles are consecutive).  Workgroup b runs on XCD
// b % 8, so XCD x is given the tile range [bin_first[x], bin_first[x + 1]),
// which its workgroups stride over: a product's tiles then share one XCD's L2
// (striding over all tiles would spread them over every XCD and fetch the same
// panels into eight caches).  The host orders and cuts the ranges (by
// estimated cost, most expensive tiles first).  Grids of fewer than 8
// workgroups stride over all tiles.
struct GroupWalk {
    int64_t t, end, stride;
    __device__ __forceinline__ explicit GroupWalk(const GroupArgs &g) {
        const int64_t G = gridDim.x, b = blockIdx.x;
        if (G < kXcds) {
            t = b;
            end = g.total_tiles;
            stride = G;
        } else {
            const int x = (int)(b % kXcds);
            t = g.bin_first[x] + b / kXcds;
            end = g.bin_first[x + 1];
            stride = (G - x + kXcds - 1) / kXcds;  // workgroups on XCD x
        }
    }
};

// Runs tile(d, local) for each tile of the workgroup's walk: d the tile's
// product, local its tile index within the product (a product's tiles fit 32
// bits).  The loads a tile's setup waits on are requested a tile early: the
// next tile's descriptor and the product index of the tile after it are
// loaded before the current tile runs (their latency otherwise opens every
// tile, and tiles here run only a few K steps).  The indices are uniform
// over the workgroup and the map and descriptors do not change while the
// kernel runs, so they are read as constants (through the scalar cache).
__device__ __forceinline__ int32_t const_load(const int32_t *p) {
    return *(const __attribute__((address_space(4))) int32_t *)p;
}

__device__ __forceinline__ GroupDesc const_load(const GroupDesc *p) {
    struct Words {
        uint32_t w[sizeof(GroupDesc) / 4];
    } v;
    static_assert(sizeof(GroupDesc) % 4 == 0, "descriptor of whole words");
    const __attribute__((address_space(4))) uint32_t *q = (const __attribute__((address_space(4))) uint32_t *)p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(GroupDesc) / 4); ++i) v.w[i] = q[i];
    return __builtin_bit_cast(GroupDesc, v);
}

template <class Tile>
__device__ __forceinline__ void walk_tiles(const GroupArgs &g, Tile &&tile) {
    GroupWalk w(g);
    if (w.t >= w.end) return;
    int gnext = const_load(g.tile_group + w.t);
    GroupDesc d = const_load(g.descs + gnext);
    if (w.t + w.stride < w.end) gnext = const_load(g.tile_group + w.t + w.stride);
    for (; w.t < w.end; w.t += w.stride) {
        const int64_t t2 = w.t + 2 * w.stride;
        const int gafter = t2 < w.end ? const_load(g.tile_group + t2) : gnext;
        const GroupDesc dn = const_load(g.descs + gnext);
        __syncthreads();  // the previous tile's LDS reads are done
        tile(d, (int)(w.t - d.tile_start));
        d = dn;
        gnext = gafter;
    }
}

// WIDE: every product of the launch has rows aligned for 16-byte loads (the
// host gives a launch only such products), so the kernel carries no
// element-load path -- fewer registers, one more resident wavefront per SIMD
// for the 64 x 64 programs; the element-load twin (WIDE = false) runs the
// products whose rows are not aligned.
template <int BM, int BN, int BK, int WM, int WN, int STAGES, bool WIDE>
__device__ __forceinline__ void grouped_f32(const GroupArgs &g) {
    using L = F32Lds<BM, BN, BK, STAGES>;
    __shared__ __attribute__((aligned(16))) float As[STAGES * L::A];
    __shared__ __attribute__((aligned(16))) float Bs[STAGES * L::B];
    walk_tiles(g, [&](const GroupDesc &d, int local) {
        const int tm = local / d.tiles_n, tn = local % d.tiles_n;
        const MmArgs a{d.A, d.B, d.C, d.lda, d.ldb, d.ldc, d.M, d.N, d.K, g.accumulate, WIDE};
        mfma_f32_tile<BM, BN, BK, WM, WN, STAGES, true>(a, tm * BM, tn * BN, WIDE, As, Bs, 0, (d.K + BK - 1) / BK);
    });
}

template <int BM, int BN, int BK, int WM, int WN, int STAGES, bool WIDE>
__device__ __forceinline__ void grouped_bf16(const GroupArgs &g) {
    using L = Bf16Lds<BM, BN, BK, STAGES>;
    __shared__ __attribute__((aligned(16))) unsigned short As[STAGES * L::A];
    __shared__ __attribute__((aligned(16))) unsigned short Bs[STAGES * L::B];
    walk_tiles(g, [&](const GroupDesc &d, int local) {
        const int tm = local / d.tiles_n, tn = local % d.tiles_n;
        const MmArgs a{d.A, d.B, d.C, d.lda, d.ldb, d.ldc, d.M, d.N, d.K, g.accumulate, WIDE};
        mfma_bf16_tile<BM, BN, BK, WM, WN, STAGES, true>(a, tm * BM, tn * BN, WIDE, As, Bs, 0, (d.K + BK - 1) / BK);
    });
}

// Mixed grouped kernels: each product's tiles run the program kMixedTile[prog]
// of its descriptor; one LDS allocation, the largest program's, serves all.
constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int STAGES> struct MixedLds {
    static constexpr int f32 =
        cmax(cmax(F32Lds<kMixedTile[0][0], kMixedTile[0][1], kMixedBk[0], STAGES>::floats,
                  F32Lds<kMixedTile[1][0], kMixedTile[1][1], kMixedBk[0], STAGES>::floats),
             cmax(F32Lds<kMixedTile[2][0], kMixedTile[2][1], kMixedBk[0], STAGES>::floats,
                  F32Lds<kMixedTile[3][0], kMixedTile[3][1], kMixedBk[0], STAGES>::floats));
    static constexpr int bf16 =
        cmax(cmax(Bf16Lds<kMixedTile[0][0], kMixedTile[0][1], kMixedBk[2], STAGES>::elems,
                  Bf16Lds<kMixedTile[1][0], kMixedTile[1][1], kMixedBk[2], STAGES>::elems),
             cmax(Bf16Lds<kMixedTile[2][0], kMixedTile[2][1], kMixedBk[2], STAGES>::elems,
                  Bf16Lds<kMixedTile[3][0], kMixedTile[3][1], kMixedBk[2], STAGES>::elems));
};

template <int P, int STAGES, bool WIDE>
__device__ __forceinline__ void mixed_f32_tile(const MmArgs &a, int local, int tiles_n, float *lds) {
    constexpr int BM = kMixedTile[P][0], BN = kMixedTile[P][1];
    const int tm = local / tiles_n, tn = local % tiles_n;
    using L = F32Lds<BM, BN, kMixedBk[0], STAGES>;
    mfma_f32_tile<BM, BN, kMixedBk[0], 2, 2, STAGES, true>(a, tm * BM, tn * BN, WIDE, lds,
                                                           lds + STAGES * L::A, 0,
                                                           (a.K + kMixedBk[0] - 1) / kMixedBk[0]);
}

template <int P, int STAGES, bool WIDE>
__device__ __forceinline__ void mixed_bf16_tile(const MmArgs &a, int local, int tiles_n, unsigned short *lds) {
    constexpr int BM = kMixedTile[P][0], BN = kMixedTile[P][1];
    const int tm = local / tiles_n, tn = local % tiles_n;
    using L = Bf16Lds<BM, BN, kMixedBk[2], STAGES>;
    mfma_bf16_tile<BM, BN, kMixedBk[2], 2, 2, STAGES, true>(a, tm * BM, tn * BN, WIDE, lds,
                                                            lds + STAGES * L::A, 0,
                                                            (a.K + kMixedBk[2] - 1) / kMixedBk[2]);
}

template <int STAGES, bool WIDE>
__device__ __forceinline__ void grouped_mixed_f32(const GroupArgs &g) {
    static_assert(kMixedPrograms == 4, "one case per program");
    __shared__ __attribute__((aligned(16))) float lds[MixedLds<STAGES>::f32];
    walk_tiles(g, [&](const GroupDesc &d, int local) {
        const MmArgs a{d.A, d.B, d.C, d.lda, d.ldb, d.ldc, d.M, d.N, d.K, g.accumulate, WIDE};
        switch (d.prog) {
        case 0: mixed_f32_tile<0, STAGES, WIDE>(a, local, d.tiles_n, lds); break;
        case 1: mixed_f32_tile<1, STAGES, WIDE>(a, local, d.tiles_n, lds); break;
        case 2: mixed_f32_tile<2, STAGES, WIDE>(a, local, d.tiles_n, lds); break;
        default: mixed_f32_tile<3, STAGES, WIDE>(a, local, d.tiles_n, lds); break;
        }
    });
}

template <int STAGES, bool WIDE>
__device__ __forceinline__ void grouped_mixed_bf16(const GroupArgs &g) {
    static_assert(kMixedPrograms == 4, "one case per program");
    __shared__ __attribute__((aligned(16))) unsigned short lds[MixedLds<STAGES>::bf16];
    walk_tiles(g, [&](const GroupDesc &d, int local) {
        const MmArgs a{d.A, d.B, d.C, d.lda, d.ldb, d.ldc, d.M, d.N, d.K, g.accumulate, WIDE};
        switch (d.prog) {
        case 0: mixed_bf16_tile<0, STAGES, WIDE>(a, local, d.tiles_n, lds); break;
        case 1: mixed_bf16_tile<1, STAGES, WIDE>(a, local, d.tiles_n, lds); break;
        case 2: mixed_bf16_tile<2, STAGES, WIDE>(a, local, d.tiles_n, lds); break;
        default: mixed_bf16_tile<3, STAGES, WIDE>(a, local, d.tiles_n, lds); break;
        }
    });
}

}  // namespace pkk
