// Parametric matrix transposition (Section 5.2, Fig. 7, Table 3), for gfx950.
//
// C (N x M) = transpose of A (M x N), 4-byte elements, row-major with leading
// dimensions.  A workgroup of B1 x B0 work-items owns a tile of (B0 * S) rows
// and B1 columns of A, i.e. every work-item moves S elements (the paper's
// granularity s).
//
// transpose_tiled (a and c cached, the paper's first case): the tile is read
//   with B1 consecutive lanes along each row of A (coalesced), stored in LDS
//   (rows padded by one element), and written with consecutive lanes along
//   each row of C (coalesced), reading LDS down a column -- the padding puts
//   those reads in distinct banks.  One barrier between the two phases; one
//   more before the tile's LDS is reused.  LDS bytes: 4 * (B0 * S) * (B1 + 1).
//   After granularity reduction (the paper's second case) S = 1.
// transpose_direct (no caching, the paper's third case): each work-item
//   copies its S elements straight from A to C (reads coalesced, writes
//   strided).
//
// The operation is pure data movement: HBM-bound, 8 bytes per element
// (one read, one write) at best.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kargs.hpp"

namespace pkk {

// Arguments of the transposition kernels: C (N x M) = A (M x N)^T.
struct TrArgs {
    const void *A;
    void *C;
    int64_t lda, ldc;
    int32_t M, N;
};

template <int B0, int B1, int S>
__device__ __forceinline__ void transpose_tiled(const TrArgs &a) {
    constexpr int NT = B0 * B1;
    constexpr int TR = B0 * S;   // tile rows (of A)
    constexpr int TC = B1;       // tile columns (of A)
    __shared__ uint32_t tile[TR][TC + 1];
    const uint32_t *__restrict__ A = static_cast<const uint32_t *>(a.A);
    uint32_t *__restrict__ C = static_cast<uint32_t *>(a.C);
    const int M = a.M, N = a.N;
    const int t = threadIdx.x;
    const int tiles_c = (N + TC - 1) / TC;
    const int64_t tiles = (int64_t)((M + TR - 1) / TR) * tiles_c;
    for (int64_t b = blockIdx.x; b < tiles; b += gridDim.x) {
        const int row0 = (int)(b / tiles_c) * TR, col0 = (int)(b % tiles_c) * TC;
        // interior tiles: no guards, so a work-item's S loads are all in
        // flight before the first LDS store waits for its data (a guard per
        // load makes each load wait for the previous one)
        const bool interior = row0 + TR <= M && col0 + TC <= N;
        if (interior) {
            uint32_t v[S];
#pragma unroll
            for (int k = 0; k < S; ++k) {  // read: lanes along a row of A
                const int e = t + k * NT;
                v[k] = A[(int64_t)(row0 + e / TC) * a.lda + col0 + e % TC];
            }
#pragma unroll
            for (int k = 0; k < S; ++k) {
                const int e = t + k * NT;
                tile[e / TC][e % TC] = v[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < S; ++k) {
                const int e = t + k * NT;
                const int r = e / TC, c = e % TC;
                const int gr = row0 + r, gc = col0 + c;
                if (gr < M && gc < N) tile[r][c] = A[(int64_t)gr * a.lda + gc];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < S; ++k) {  // write: lanes along a row of C
            const int e = t + k * NT;
            const int cr = e / TR, cc = e % TR;  // C row = A column, C column = A row
            const int gr = col0 + cr, gc = row0 + cc;
            if (interior || (gr < N && gc < M)) C[(int64_t)gr * a.ldc + gc] = tile[cc][cr];
        }
        __syncthreads();
    }
}

template <int B0, int B1, int S>
__device__ __forceinline__ void transpose_direct(const TrArgs &a) {
    constexpr int NT = B0 * B1;
    constexpr int TR = B0 * S;
    constexpr int TC = B1;
    const uint32_t *__restrict__ A = static_cast<const uint32_t *>(a.A);
    uint32_t *__restrict__ C = static_cast<uint32_t *>(a.C);
    const int M = a.M, N = a.N;
    const int t = threadIdx.x;
    const int tiles_c = (N + TC - 1) / TC;
    const int64_t tiles = (int64_t)((M + TR - 1) / TR) * tiles_c;
    for (int64_t b = blockIdx.x; b < tiles; b += gridDim.x) {
        const int row0 = (int)(b / tiles_c) * TR, col0 = (int)(b % tiles_c) * TC;
        if (row0 + TR <= M && col0 + TC <= N) {  // interior: loads in flight together
            uint32_t v[S];
#pragma unroll
            for (int k = 0; k < S; ++k) {
                const int e = t + k * NT;
                v[k] = A[(int64_t)(row0 + e / TC) * a.lda + col0 + e % TC];
            }
#pragma unroll
            for (int k = 0; k < S; ++k) {
                const int e = t + k * NT;
                C[(int64_t)(col0 + e % TC) * a.ldc + row0 + e / TC] = v[k];
            }
            continue;
        }
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const int e = t + k * NT;
            const int r = e / TC, c = e % TC;
            const int gr = row0 + r, gc = col0 + c;
            if (gr < M && gc < N) C[(int64_t)gc * a.ldc + gr] = A[(int64_t)gr * a.lda + gc];
        }
    }
}

}  // namespace pkk
