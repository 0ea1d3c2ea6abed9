// VALU kernels of the blocked matrix product (Section 2, Fig. 3 and Fig. 4),
// written for gfx950.
//
// Work decomposition (Fig. 3): a workgroup of BX x BY work-items owns an
// output tile of BY rows and BX*S columns.  Work-item (ty, tx) computes the S
// outputs C[row0 + ty][col0 + tx + w*BX], w < S, so consecutive lanes write
// consecutive columns (coalesced, as the paper notes for its a, b, c accesses).
// Tiles are visited with a workgroup-stride loop over the linear tile index
// (the paper strides its blocks by a fixed 256; here the stride is the grid).
//
// valu_tiled (no strategy applied; or at S = 1 after granularity reduction):
//   per K step of BK, the workgroup stages the A tile (BY x BK) and the B tile
//   (BK x BX*S) in LDS with cooperative, coalesced loads (zero fill outside
//   the matrices), synchronises, accumulates from LDS, synchronises again --
//   the two barriers per K tile of Fig. 4.  The A tile rows are padded by one
//   element so the BY rows a wavefront reads at the same k fall in different
//   banks.  LDS bytes: esize * (BY * (BK + 1) + BK * BX * S).
// valu_direct (decision (4b), no LDS): every work-item reads its A row and B
//   columns from global memory (the A element is common to the lanes of a
//   row, the B elements are contiguous across lanes).
//
// Arithmetic: float32 accumulates with fused multiply-add in k order starting
// from C (accumulate) or 0; int32 accumulates in uint32, i.e. modulo 2^32.
// Any M, N, K >= 0 is handled: loads are guarded and stores are guarded.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kargs.hpp"

namespace pkk {

template <typename T> struct Acc;
template <> struct Acc<float> {
    using type = float;
    static __device__ __forceinline__ float from(float x) { return x; }
    static __device__ __forceinline__ float to(float x) { return x; }
    static __device__ __forceinline__ float mad(float acc, float a, float b) { return __builtin_fmaf(a, b, acc); }
};
template <> struct Acc<int32_t> {
    using type = uint32_t;
    static __device__ __forceinline__ uint32_t from(int32_t x) { return (uint32_t)x; }
    static __device__ __forceinline__ int32_t to(uint32_t x) { return (int32_t)x; }
    static __device__ __forceinline__ uint32_t mad(uint32_t acc, uint32_t a, uint32_t b) { return acc + a * b; }
};

template <typename T, int BX, int BY, int S, int BK>
__device__ __forceinline__ void valu_tiled(const MmArgs &a) {
    using U = typename Acc<T>::type;
    constexpr int NT = BX * BY;
    constexpr int TM = BY;
    constexpr int TN = BX * S;
    __shared__ T As[TM][BK + 1];
    __shared__ T Bs[BK][TN];

    const T *__restrict__ A = static_cast<const T *>(a.A);
    const T *__restrict__ B = static_cast<const T *>(a.B);
    T *__restrict__ C = static_cast<T *>(a.C);
    const int M = a.M, N = a.N, K = a.K;
    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int tiles_n = (N + TN - 1) / TN;
    const int64_t tiles = (int64_t)((M + TM - 1) / TM) * tiles_n;

    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int row0 = (int)(t / tiles_n) * TM;
        const int col0 = (int)(t % tiles_n) * TN;
        const int row = row0 + ty;
        U acc[S];
#pragma unroll
        for (int w = 0; w < S; ++w) {
            const int col = col0 + tx + w * BX;
            acc[w] = (a.accumulate && row < M && col < N) ? Acc<T>::from(C[(int64_t)row * a.ldc + col]) : U(0);
        }
        constexpr int UA = (TM * BK + NT - 1) / NT, UB = (BK * TN + NT - 1) / NT;
        const bool inside = row0 + TM <= M && col0 + TN <= N;
        for (int k0 = 0; k0 < K; k0 += BK) {
            if (inside && k0 + BK <= K) {
                // the whole K tile in range: no guards, so a work-item's loads
                // are all in flight before the first LDS store waits (a guard
                // per load makes each wait for the one before)
                T va[UA], vb[UB];
#pragma unroll
                for (int u = 0; u < UA; ++u) {
                    const int e = tid + u * NT;
                    if ((TM * BK) % NT == 0 || e < TM * BK)
                        va[u] = A[(int64_t)(row0 + e / BK) * a.lda + k0 + e % BK];
                }
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const int e = tid + u * NT;
                    if ((BK * TN) % NT == 0 || e < BK * TN)
                        vb[u] = B[(int64_t)(k0 + e / TN) * a.ldb + col0 + e % TN];
                }
#pragma unroll
                for (int u = 0; u < UA; ++u) {
                    const int e = tid + u * NT;
                    if ((TM * BK) % NT == 0 || e < TM * BK) As[e / BK][e % BK] = va[u];
                }
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const int e = tid + u * NT;
                    if ((BK * TN) % NT == 0 || e < BK * TN) Bs[e / TN][e % TN] = vb[u];
                }
                __syncthreads();
#pragma unroll
                for (int kk = 0; kk < BK; ++kk) {
                    const U av = (U)As[ty][kk];
#pragma unroll
                    for (int w = 0; w < S; ++w) acc[w] = Acc<T>::mad(acc[w], av, (U)Bs[kk][tx + w * BX]);
                }
                __syncthreads();
                continue;
            }
#pragma unroll
            for (int u = 0; u < (TM * BK + NT - 1) / NT; ++u) {
                const int e = tid + u * NT;
                if ((TM * BK) % NT == 0 || e < TM * BK) {
                    const int r = e / BK, c = e % BK;
                    const int gr = row0 + r, gc = k0 + c;
                    As[r][c] = (gr < M && gc < K) ? A[(int64_t)gr * a.lda + gc] : T(0);
                }
            }
#pragma unroll
            for (int u = 0; u < (BK * TN + NT - 1) / NT; ++u) {
                const int e = tid + u * NT;
                if ((BK * TN) % NT == 0 || e < BK * TN) {
                    const int r = e / TN, c = e % TN;
                    const int gr = k0 + r, gc = col0 + c;
                    Bs[r][c] = (gr < K && gc < N) ? B[(int64_t)gr * a.ldb + gc] : T(0);
                }
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < BK; ++kk) {
                const U av = (U)As[ty][kk];
#pragma unroll
                for (int w = 0; w < S; ++w) acc[w] = Acc<T>::mad(acc[w], av, (U)Bs[kk][tx + w * BX]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int w = 0; w < S; ++w) {
            const int col = col0 + tx + w * BX;
            if (row < M && col < N) C[(int64_t)row * a.ldc + col] = Acc<T>::to(acc[w]);
        }
    }
}

// valu_tiled2 (the 2-D micro-tile program, Fig. 4's kernel with outputs per
// work-item along M as well): a workgroup of BX x BY work-items owns a tile
// of BY * SY rows and BX * SX columns; work-item (ty, tx) computes the outputs
// at rows row0 + ty + v * BY (v < SY) and the SX consecutive columns
// col0 + tx * SX + w (w < SX), so a workgroup's store of one row is still one
// contiguous run.  The LDS tiles are the A tile (BY * SY) x BK, rows padded to
// BK + 4 elements (16-byte aligned rows; the rows one wavefront reads start
// four banks apart), and the B tile BK x (BX * SX), with a K extent BK of its
// own.  Per four k a work-item reads SY 16-byte words of A (four k of one row;
// shared by the BX work-items of that row) and four SX-element words of B
// (contiguous across the lanes), for 4 * SY * SX multiply-adds: the paper's
// program (SY = 1, one element per read) reads 1 + S elements per S.  Each
// output sums k in ascending order, as the one-row program does.
template <typename T, int BX, int BY, int SX, int SY, int BK>
__device__ __forceinline__ void valu_tiled2(const MmArgs &a) {
    using U = typename Acc<T>::type;
    constexpr int NT = BX * BY;
    constexpr int TM = BY * SY;
    constexpr int TN = BX * SX;
    constexpr int LDA = BK + 4;
    static_assert(BK % 4 == 0, "K tile of whole 16-byte words");
    static_assert(SX == 1 || SX == 2 || SX == 4, "B words of 1, 2 or 4 elements");
    __shared__ __attribute__((aligned(16))) T As[TM][LDA];
    __shared__ __attribute__((aligned(16))) T Bs[BK][TN];
    typedef T t4 __attribute__((ext_vector_type(4)));
    typedef T tsx __attribute__((ext_vector_type(SX == 1 ? 2 : SX)));  // SX == 1 reads one element

    const T *__restrict__ A = static_cast<const T *>(a.A);
    const T *__restrict__ B = static_cast<const T *>(a.B);
    T *__restrict__ C = static_cast<T *>(a.C);
    const int M = a.M, N = a.N, K = a.K;
    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int tiles_n = (N + TN - 1) / TN;
    const int64_t tiles = (int64_t)((M + TM - 1) / TM) * tiles_n;
    constexpr int UA = (TM * BK + NT - 1) / NT, UB = (BK * TN + NT - 1) / NT;

    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int row0 = (int)(t / tiles_n) * TM;
        const int col0 = (int)(t % tiles_n) * TN;
        U acc[SY][SX];
#pragma unroll
        for (int v = 0; v < SY; ++v)
#pragma unroll
            for (int w = 0; w < SX; ++w) {
                const int row = row0 + ty + v * BY, col = col0 + tx * SX + w;
                acc[v][w] = (a.accumulate && row < M && col < N) ? Acc<T>::from(C[(int64_t)row * a.ldc + col]) : U(0);
            }
        const bool inside = row0 + TM <= M && col0 + TN <= N;
        for (int k0 = 0; k0 < K; k0 += BK) {
            if (inside && k0 + BK <= K) {
                // the whole K tile in range: unguarded loads, all in flight
                // before the first LDS store
                T va[UA], vb[UB];
#pragma unroll
                for (int u = 0; u < UA; ++u) {
                    const int e = tid + u * NT;
                    if ((TM * BK) % NT == 0 || e < TM * BK)
                        va[u] = A[(int64_t)(row0 + e / BK) * a.lda + k0 + e % BK];
                }
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const int e = tid + u * NT;
                    if ((BK * TN) % NT == 0 || e < BK * TN)
                        vb[u] = B[(int64_t)(k0 + e / TN) * a.ldb + col0 + e % TN];
                }
#pragma unroll
                for (int u = 0; u < UA; ++u) {
                    const int e = tid + u * NT;
                    if ((TM * BK) % NT == 0 || e < TM * BK) As[e / BK][e % BK] = va[u];
                }
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const int e = tid + u * NT;
                    if ((BK * TN) % NT == 0 || e < BK * TN) Bs[e / TN][e % TN] = vb[u];
                }
            } else {
#pragma unroll
                for (int u = 0; u < UA; ++u) {
                    const int e = tid + u * NT;
                    if ((TM * BK) % NT == 0 || e < TM * BK) {
                        const int r = e / BK, c = e % BK;
                        const int gr = row0 + r, gc = k0 + c;
                        As[r][c] = (gr < M && gc < K) ? A[(int64_t)gr * a.lda + gc] : T(0);
                    }
                }
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const int e = tid + u * NT;
                    if ((BK * TN) % NT == 0 || e < BK * TN) {
                        const int r = e / TN, c = e % TN;
                        const int gr = k0 + r, gc = col0 + c;
                        Bs[r][c] = (gr < K && gc < N) ? B[(int64_t)gr * a.ldb + gc] : T(0);
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                t4 av[SY];
                U bv[4][SX];
#pragma unroll
                for (int v = 0; v < SY; ++v) av[v] = *reinterpret_cast<const t4 *>(&As[ty + v * BY][kk]);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if constexpr (SX == 1) {
                        bv[q][0] = (U)Bs[kk + q][tx];
                    } else {
                        const tsx b = *reinterpret_cast<const tsx *>(&Bs[kk + q][tx * SX]);
#pragma unroll
                        for (int w = 0; w < SX; ++w) bv[q][w] = (U)b[w];
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int v = 0; v < SY; ++v)
#pragma unroll
                        for (int w = 0; w < SX; ++w) acc[v][w] = Acc<T>::mad(acc[v][w], (U)av[v][q], bv[q][w]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int v = 0; v < SY; ++v)
#pragma unroll
            for (int w = 0; w < SX; ++w) {
                const int row = row0 + ty + v * BY, col = col0 + tx * SX + w;
                if (row < M && col < N) C[(int64_t)row * a.ldc + col] = Acc<T>::to(acc[v][w]);
            }
    }
}

template <typename T, int BX, int BY, int S>
__device__ __forceinline__ void valu_direct(const MmArgs &a) {
    using U = typename Acc<T>::type;
    constexpr int TM = BY;
    constexpr int TN = BX * S;
    const T *__restrict__ A = static_cast<const T *>(a.A);
    const T *__restrict__ B = static_cast<const T *>(a.B);
    T *__restrict__ C = static_cast<T *>(a.C);
    const int M = a.M, N = a.N, K = a.K;
    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int tiles_n = (N + TN - 1) / TN;
    const int64_t tiles = (int64_t)((M + TM - 1) / TM) * tiles_n;

    for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int row = (int)(t / tiles_n) * TM + ty;
        const int col0 = (int)(t % tiles_n) * TN + tx;
        if (row >= M) continue;
        U acc[S];
#pragma unroll
        for (int w = 0; w < S; ++w) {
            const int col = col0 + w * BX;
            acc[w] = (a.accumulate && col < N) ? Acc<T>::from(C[(int64_t)row * a.ldc + col]) : U(0);
        }
        const T *arow = A + (int64_t)row * a.lda;
        for (int k = 0; k < K; ++k) {
            const U av = (U)arow[k];
            const T *brow = B + (int64_t)k * a.ldb;
#pragma unroll
            for (int w = 0; w < S; ++w) {
                const int col = col0 + w * BX;
                const U bv = col < N ? (U)brow[col] : U(0);
                acc[w] = Acc<T>::mad(acc[w], av, bv);
            }
        }
#pragma unroll
        for (int w = 0; w < S; ++w) {
            const int col = col0 + w * BX;
            if (col < N) C[(int64_t)row * a.ldc + col] = Acc<T>::to(acc[w]);
        }
    }
}

}  // namespace pkk
