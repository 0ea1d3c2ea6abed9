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
//   bfloat16: As[BM][BK+8]   (k contiguous),   Bt[BN][BK+8]   (B transposed,
//             k contiguous, so each lane reads its 8 k values with one 16-byte
//             LDS load)
// STAGES = 2 double-buffers the tiles (one barrier per K step: the next tile is
// fetched from global memory into registers while the current one is
// consumed); STAGES = 1 keeps one buffer and two barriers per step, as in the
// paper's kernel.  LDS bytes = STAGES * (A tile + B tile).
//
// The order in which k enters each 32x32 block's sum is permuted: lanes 0-31
// consume k in the first half of the LDS tile and lanes 32-63 the second half,
// so a lane's operands are contiguous in LDS.  The set of products summed is
// unchanged.
//
// Global loads are 16 bytes wide, so the leading dimensions must keep rows
// 16-byte aligned (lda, ldb multiples of 4 floats / 8 bfloat16 and 16-byte
// aligned bases); the host checks this.  Tiles crossing the matrix edge clamp
// the rows of A and the columns of B they read to the last one in range
// (results outside C are never stored), read k beyond K from a block of zeros,
// and guard their stores.  Edge loads choose an address, never a loaded value,
// so they carry no branches and stay in flight together.
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

constexpr int XCDS = 8;
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
// One BM x BN output tile at (row0, col0).  `vec`: the rows of A and B are
// 16-byte aligned, so interior tiles may use 16-byte loads.  The caller
// synchronises the workgroup before reusing the LDS for another tile.
template <int BM, int BN, int BK, int WM, int WN, int STAGES, bool EDGE_ADDR>
__device__ __forceinline__ void mfma_f32_tile(const MmArgs &a, const int row0, const int col0, const bool vec) {
    constexpr int NT = 64 * WM * WN;
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 32, TN = WTN / 32;
    constexpr int PA = 4, PB = 4;
    constexpr int LDA_S = BK + PA, LDB_S = BN + PB;
    constexpr int A4 = BM * BK / 4 / NT;  // float4 loads per work-item per A tile
    constexpr int B4 = BK * BN / 4 / NT;
    static_assert(TM >= 1 && TN >= 1 && WTM % 32 == 0 && WTN % 32 == 0, "wave tile must be 32x32 blocks");
    static_assert(A4 >= 1 && B4 >= 1 && (BM * BK / 4) % NT == 0 && (BK * BN / 4) % NT == 0, "tile loads");
    static_assert(BK % 8 == 0, "BK");

    __shared__ __attribute__((aligned(16))) float As[STAGES][BM * LDA_S];
    __shared__ __attribute__((aligned(16))) float Bs[STAGES][BK * LDB_S];

    const gptr<float> __restrict__ A = (gptr<float>)a.A;
    const gptr<float> __restrict__ B = (gptr<float>)a.B;
    const gmut<float> __restrict__ C = (gmut<float>)a.C;
    const int M = a.M, N = a.N, K = a.K;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int r = lane & 31, h = lane >> 5;

    const bool interior = (row0 + BM <= M) && (col0 + BN <= N);

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
    // Any K step, edge tiles included.  EDGE_ADDR: every load goes to a chosen
    // address (the wide/narrow choices are uniform across the workgroup), for
    // programs whose steps are mostly edge steps (element loads, many small
    // products); otherwise guarded loads, which hold fewer registers where
    // edge steps are rare.
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
        if (vec && k0 + BK <= K) {
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
                const gptr<float> row = A + (int64_t)min(row0 + rr, M - 1) * a.lda;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = k0 + c4 + e;
                    ra[u][e] = *(k < K ? row + k : zero);
                }
            }
        }
        if (vec && col0 + BN <= N) {
#pragma unroll
            for (int u = 0; u < B4; ++u) {
                const int f = tid + u * NT;
                const int rr = f / (BN / 4), c4 = (f % (BN / 4)) * 4;
                const int k = k0 + rr;
                rb[u] = *reinterpret_cast<gptr<f32x4>>(k < K ? B + (int64_t)k * a.ldb + col0 + c4 : zero);
            }
        } else {
#pragma unroll
            for (int u = 0; u < B4; ++u) {
                const int f = tid + u * NT;
                const int rr = f / (BN / 4), c4 = (f % (BN / 4)) * 4;
                const int k = k0 + rr;
                const gptr<float> row = k < K ? B + (int64_t)k * a.ldb : nullptr;
#pragma unroll
                for (int e = 0; e < 4; ++e) rb[u][e] = *(row ? row + min(col0 + c4 + e, N - 1) : zero);
            }
        }
    };
    auto sstore = [&](int st) {
#pragma unroll
        for (int u = 0; u < A4; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BK / 4), c4 = (f % (BK / 4)) * 4;
            *reinterpret_cast<f32x4 *>(&As[st][rr * LDA_S + c4]) = ra[u];
        }
#pragma unroll
        for (int u = 0; u < B4; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BN / 4), c4 = (f % (BN / 4)) * 4;
            *reinterpret_cast<f32x4 *>(&Bs[st][rr * LDB_S + c4]) = rb[u];
        }
    };
    auto compute = [&](int st) {
        const float *as = &As[st][(wm * WTM + r) * LDA_S + h * (BK / 2)];
        const float *bs = &Bs[st][(h * (BK / 2)) * LDB_S + wn * WTN + r];
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

    const int KT = (K + BK - 1) / BK;
    // leading K steps that need no guards: all of them for an interior tile
    // on aligned rows, except a partial last one
    const int KF = (vec && interior) ? K / BK : 0;
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
            compute(cur);
            sstore(cur ^ 1);
            __syncthreads();
        }
        for (; kt < KT; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < KT) gload((kt + 1) * BK);
            compute(cur);
            if (kt + 1 < KT) sstore(cur ^ 1);
            __syncthreads();
        }
    } else {
        int kt = 0;
        for (; kt < KF; ++kt) {
            gload_fast(kt * BK);
            __syncthreads();
            sstore(0);
            __syncthreads();
            compute(0);
        }
        for (; kt < KT; ++kt) {
            gload(kt * BK);
            __syncthreads();
            sstore(0);
            __syncthreads();
            compute(0);
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
                    *p = a.accumulate ? *p + acc[i][j][v] : acc[i][j][v];
                }
            }
        }
}

// ------------------------------------------------------------------ bfloat16
// bfloat16 tile; `vec`: A rows 16-byte aligned and B rows 4-byte aligned.
template <int BM, int BN, int BK, int WM, int WN, int STAGES, bool EDGE_ADDR>
__device__ __forceinline__ void mfma_bf16_tile(const MmArgs &a, const int row0, const int col0, const bool vec) {
    constexpr int NT = 64 * WM * WN;
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 32, TN = WTN / 32;
    constexpr int P = 8;
    constexpr int LD_S = BK + P;                 // row stride (elements) of As and Bt
    constexpr int A8 = BM * BK / 8 / NT;         // 16-byte loads per work-item per A tile
    constexpr int B8 = (BK / 8) * (BN / 2) / NT; // (8 k rows x 2 columns) blocks per work-item
    static_assert(TM >= 1 && TN >= 1 && WTM % 32 == 0 && WTN % 32 == 0, "wave tile must be 32x32 blocks");
    static_assert(A8 >= 1 && B8 >= 1 && (BM * BK / 8) % NT == 0 && ((BK / 8) * (BN / 2)) % NT == 0, "tile loads");
    static_assert(BK % 32 == 0, "BK");

    __shared__ __attribute__((aligned(16))) unsigned short As[STAGES][BM * LD_S];
    __shared__ __attribute__((aligned(16))) unsigned short Bt[STAGES][BN * LD_S];

    const gptr<unsigned short> __restrict__ A = (gptr<unsigned short>)a.A;
    const gptr<unsigned short> __restrict__ B = (gptr<unsigned short>)a.B;
    const gmut<float> __restrict__ C = (gmut<float>)a.C;
    const int M = a.M, N = a.N, K = a.K;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int r = lane & 31, h = lane >> 5;

    const bool interior = (row0 + BM <= M) && (col0 + BN <= N);

    f32x16 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

    u16x8 ra[A8];
    unsigned int rb[B8][8];  // 8 k rows of a column pair (n, n+1)
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
            const int cp = (f % (BN / 2)) * 2, kr = (f / (BN / 2)) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                rb[u][e] = *reinterpret_cast<gptr<unsigned int>>(B + (int64_t)(k0 + kr + e) * a.ldb + col0 + cp);
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
                const int cp = (f % (BN / 2)) * 2, kr = (f / (BN / 2)) * 8;
                const int gc = col0 + cp;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int gr = k0 + kr + e;
                    if (vec && gr < K && gc + 2 <= N) {
                        rb[u][e] = *reinterpret_cast<gptr<unsigned int>>(B + (int64_t)gr * a.ldb + gc);
                    } else {
                        const unsigned int lo = (gr < K && gc < N) ? B[(int64_t)gr * a.ldb + gc] : 0u;
                        const unsigned int hi = (gr < K && gc + 1 < N) ? B[(int64_t)gr * a.ldb + gc + 1] : 0u;
                        rb[u][e] = lo | (hi << 16);
                    }
                }
            }
            return;
        }
        if (vec && k0 + BK <= K) {
#pragma unroll
            for (int u = 0; u < A8; ++u) {
                const int f = tid + u * NT;
                const int rr = f / (BK / 8), c8 = (f % (BK / 8)) * 8;
                ra[u] = *reinterpret_cast<gptr<u16x8>>(A + (int64_t)min(row0 + rr, M - 1) * a.lda + k0 + c8);
            }
        } else {
            const gptr<unsigned short> zero = (gptr<unsigned short>)(const void *)kZeroBlock;
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
        }
        if (vec && col0 + BN <= N) {
#pragma unroll
            for (int u = 0; u < B8; ++u) {
                const int f = tid + u * NT;
                const int cp = (f % (BN / 2)) * 2, kr = (f / (BN / 2)) * 8;  // column pair, first k row
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = k0 + kr + e;
                    rb[u][e] = *(k < K ? reinterpret_cast<gptr<unsigned int>>(B + (int64_t)k * a.ldb + col0 + cp)
                                       : (gptr<unsigned int>)(const void *)kZeroBlock);
                }
            }
        } else {
            const gptr<unsigned short> zero = (gptr<unsigned short>)(const void *)kZeroBlock;
#pragma unroll
            for (int u = 0; u < B8; ++u) {
                const int f = tid + u * NT;
                const int cp = (f % (BN / 2)) * 2, kr = (f / (BN / 2)) * 8;
                const int c0 = min(col0 + cp, N - 1), c1 = min(col0 + cp + 1, N - 1);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = k0 + kr + e;
                    const gptr<unsigned short> row = k < K ? B + (int64_t)k * a.ldb : nullptr;
                    const unsigned int lo = *(row ? row + c0 : zero), hi = *(row ? row + c1 : zero);
                    rb[u][e] = lo | (hi << 16);
                }
            }
        }
    };
    auto sstore = [&](int st) {
#pragma unroll
        for (int u = 0; u < A8; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BK / 8), c8 = (f % (BK / 8)) * 8;
            *reinterpret_cast<u16x8 *>(&As[st][rr * LD_S + c8]) = ra[u];
        }
#pragma unroll
        for (int u = 0; u < B8; ++u) {
            const int f = tid + u * NT;
            const int cp = (f % (BN / 2)) * 2, kr = (f / (BN / 2)) * 8;
            u32x4 lo, hi;  // column cp and cp + 1, 8 k values each
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const unsigned int w0 = rb[u][2 * e], w1 = rb[u][2 * e + 1];
                lo[e] = (w0 & 0xffffu) | (w1 << 16);
                hi[e] = (w0 >> 16) | (w1 & 0xffff0000u);
            }
            *reinterpret_cast<u32x4 *>(&Bt[st][cp * LD_S + kr]) = lo;
            *reinterpret_cast<u32x4 *>(&Bt[st][(cp + 1) * LD_S + kr]) = hi;
        }
    };
    auto compute = [&](int st) {
        const unsigned short *as = &As[st][(wm * WTM + r) * LD_S + h * (BK / 2)];
        const unsigned short *bs = &Bt[st][(wn * WTN + r) * LD_S + h * (BK / 2)];
#pragma unroll
        for (int kc = 0; kc < BK / 2; kc += 8) {
            bf16x8 af[TM], bf[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) af[i] = *reinterpret_cast<const bf16x8 *>(as + i * 32 * LD_S + kc);
#pragma unroll
            for (int j = 0; j < TN; ++j) bf[j] = *reinterpret_cast<const bf16x8 *>(bs + j * 32 * LD_S + kc);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
    };

    const int KT = (K + BK - 1) / BK;
    // leading K steps that need no guards: all of them for an interior tile
    // on aligned rows, except a partial last one
    const int KF = (vec && interior) ? K / BK : 0;
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
            compute(cur);
            sstore(cur ^ 1);
            __syncthreads();
        }
        for (; kt < KT; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < KT) gload((kt + 1) * BK);
            compute(cur);
            if (kt + 1 < KT) sstore(cur ^ 1);
            __syncthreads();
        }
    } else {
        int kt = 0;
        for (; kt < KF; ++kt) {
            gload_fast(kt * BK);
            __syncthreads();
            sstore(0);
            __syncthreads();
            compute(0);
        }
        for (; kt < KT; ++kt) {
            gload(kt * BK);
            __syncthreads();
            sstore(0);
            __syncthreads();
            compute(0);
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
                    *p = a.accumulate ? *p + acc[i][j][v] : acc[i][j][v];
                }
            }
        }
}

// ------------------------------------------------------------------ single product
// WIDE: 16-byte loads along aligned rows; the element-load twin (WIDE =
// false) is a kernel of its own, so neither carries the other's load path.
// The twins of workgroups up to 256 work-items load at chosen addresses (all
// their steps take the edge path).
template <int BM, int BN, int BK, int WM, int WN, int STAGES, bool WIDE = true>
__device__ __forceinline__ void mfma_f32(const MmArgs &a) {
    int tm, tn;
    tile_of(blockIdx.x, (a.M + BM - 1) / BM, (a.N + BN - 1) / BN, &tm, &tn);
    mfma_f32_tile<BM, BN, BK, WM, WN, STAGES, !WIDE && WM * WN < 8>(a, tm * BM, tn * BN, WIDE);
}

template <int BM, int BN, int BK, int WM, int WN, int STAGES, bool WIDE = true>
__device__ __forceinline__ void mfma_bf16(const MmArgs &a) {
    int tm, tn;
    tile_of(blockIdx.x, (a.M + BM - 1) / BM, (a.N + BN - 1) / BN, &tm, &tn);
    mfma_bf16_tile<BM, BN, BK, WM, WN, STAGES, !WIDE && WM * WN < 8>(a, tm * BM, tn * BN, WIDE);
}

// ------------------------------------------------------------------ grouped (persistent)
// Many independent products in one launch; tile t belongs to group
// tile_group[t] and is tile t - tile_start of that group, numbered row-major
// over its tiles (a product's tiles are consecutive).  Workgroup b runs on XCD
// b % 8, so XCD x is given the contiguous tile range [x T / 8, (x + 1) T / 8),
// which its workgroups stride over: a product's tiles then share one XCD's L2
// (striding over all tiles would spread them over every XCD and fetch the same
// panels into eight caches).  Grids of fewer than 8 workgroups stride over all
// tiles.
struct GroupWalk {
    int64_t t, end, stride;
    __device__ __forceinline__ explicit GroupWalk(int64_t total) {
        const int64_t G = gridDim.x, b = blockIdx.x;
        if (G < XCDS) {
            t = b;
            end = total;
            stride = G;
        } else {
            const int64_t x = b % XCDS;
            t = total * x / XCDS + b / XCDS;
            end = total * (x + 1) / XCDS;
            stride = (G - x + XCDS - 1) / XCDS;  // workgroups on XCD x
        }
    }
};

template <int BM, int BN, int BK, int WM, int WN, int STAGES>
__device__ __forceinline__ void grouped_f32(const GroupArgs &g) {
    for (GroupWalk w(g.total_tiles); w.t < w.end; w.t += w.stride) {
        const GroupDesc &d = g.descs[g.tile_group[w.t]];
        const int64_t local = w.t - d.tile_start;
        const int tm = (int)(local / d.tiles_n), tn = (int)(local % d.tiles_n);
        const MmArgs a{d.A, d.B, d.C, d.lda, d.ldb, d.ldc, d.M, d.N, d.K, g.accumulate, d.vec};
        __syncthreads();  // the previous tile's LDS reads are done
        mfma_f32_tile<BM, BN, BK, WM, WN, STAGES, true>(a, tm * BM, tn * BN, d.vec != 0);
    }
}

template <int BM, int BN, int BK, int WM, int WN, int STAGES>
__device__ __forceinline__ void grouped_bf16(const GroupArgs &g) {
    for (GroupWalk w(g.total_tiles); w.t < w.end; w.t += w.stride) {
        const GroupDesc &d = g.descs[g.tile_group[w.t]];
        const int64_t local = w.t - d.tile_start;
        const int tm = (int)(local / d.tiles_n), tn = (int)(local % d.tiles_n);
        const MmArgs a{d.A, d.B, d.C, d.lda, d.ldb, d.ldc, d.M, d.N, d.K, g.accumulate, d.vec};
        __syncthreads();
        mfma_bf16_tile<BM, BN, BK, WM, WN, STAGES, true>(a, tm * BM, tn * BN, d.vec != 0);
    }
}

}  // namespace pkk
