// Parametric matrix addition (Section 1, Fig. 1 and Fig. 2), for gfx950.
//
// C = A + B for M x N row-major matrices with leading dimensions.  A
// workgroup of BX x BY work-items owns BY rows and BX * S columns; work-item
// (ty, tx) adds S elements of row ty, the lanes of a wavefront touching
// consecutive addresses (Fig. 2's K1 adds the two elements j and j + N/2 of
// a row; here the S elements of a thread are BX apart, or, when rows are
// 16-byte aligned, S / VW groups of VW consecutive elements BX groups apart,
// VW = 4 or 2 -- one wide access per group).  After granularity reduction
// (Fig. 2's K2) S = 1.  int32 adds modulo 2^32; float32 adds with
// one rounding.  No LDS: the only resources are registers and work-items.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pkk {

struct MaArgs {
    const void *A;
    const void *B;
    void *C;
    int64_t lda, ldb, ldc;
    int32_t M, N;
    int32_t vec;  // rows 16-byte aligned: A, B, C aligned and every leading dimension a multiple of 4
};

template <typename T> struct AddOp;
template <> struct AddOp<float> {
    using bits = float;
    static __device__ __forceinline__ float add(float a, float b) { return a + b; }
};
template <> struct AddOp<int32_t> {
    using bits = uint32_t;  // wrapping arithmetic
    static __device__ __forceinline__ int32_t add(int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); }
};

template <typename E, int W> using vec_of = E __attribute__((ext_vector_type(W)));

// VW consecutive elements per access (VW = 1: the paper's element accesses).
// With VW > 1 a work-item's S elements are S / VW groups of VW, the groups
// BX apart, so a wavefront still covers one contiguous row segment.
template <typename T, int BX, int BY, int S, int VW>
__device__ __forceinline__ void madd_body(const MaArgs &a) {
    using E = typename AddOp<T>::bits;
    using V = vec_of<E, VW>;
    constexpr int TN = BX * S, G = S / VW;
    const E *__restrict__ A = static_cast<const E *>(a.A);
    const E *__restrict__ B = static_cast<const E *>(a.B);
    E *__restrict__ C = static_cast<E *>(a.C);
    const int M = a.M, N = a.N;
    const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
    const int tiles_n = (N + TN - 1) / TN;
    const int64_t tiles = (int64_t)((M + BY - 1) / BY) * tiles_n;
    for (int64_t b = blockIdx.x; b < tiles; b += gridDim.x) {
        const int row = (int)(b / tiles_n) * BY + ty;
        const int col0 = (int)(b % tiles_n) * TN;
        if (row >= M) continue;
        const E *ar = A + (int64_t)row * a.lda;
        const E *br = B + (int64_t)row * a.ldb;
        E *cr = C + (int64_t)row * a.ldc;
        V va[G], vb[G];
        // the whole row segment in range: no guards, so a work-item's G loads
        // are in flight together (one group needs no such path)
        if (G > 1 && col0 + TN <= N) {
#pragma unroll
            for (int w = 0; w < G; ++w) {
                const int col = col0 + (tx + w * BX) * VW;
                va[w] = *reinterpret_cast<const V *>(ar + col);
                vb[w] = *reinterpret_cast<const V *>(br + col);
            }
#pragma unroll
            for (int w = 0; w < G; ++w) {
                const int col = col0 + (tx + w * BX) * VW;
                V vc;
#pragma unroll
                for (int e = 0; e < VW; ++e) vc[e] = (E)AddOp<T>::add((T)va[w][e], (T)vb[w][e]);
                *reinterpret_cast<V *>(cr + col) = vc;
            }
            continue;
        }
#pragma unroll
        for (int w = 0; w < G; ++w) {
            const int col = col0 + (tx + w * BX) * VW;
            if (col + VW <= N) {
                va[w] = *reinterpret_cast<const V *>(ar + col);
                vb[w] = *reinterpret_cast<const V *>(br + col);
            } else {
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    va[w][e] = col + e < N ? ar[col + e] : E(0);
                    vb[w][e] = col + e < N ? br[col + e] : E(0);
                }
            }
        }
#pragma unroll
        for (int w = 0; w < G; ++w) {
            const int col = col0 + (tx + w * BX) * VW;
            V vc;
#pragma unroll
            for (int e = 0; e < VW; ++e) vc[e] = (E)AddOp<T>::add((T)va[w][e], (T)vb[w][e]);
            if (col + VW <= N) {
                *reinterpret_cast<V *>(cr + col) = vc;
            } else {
#pragma unroll
                for (int e = 0; e < VW; ++e)
                    if (col + e < N) cr[col + e] = vc[e];
            }
        }
    }
}

template <typename T, int BX, int BY, int S>
__device__ __forceinline__ void madd(const MaArgs &a) {
    constexpr int VW = (S % 4 == 0) ? 4 : (S % 2 == 0 ? 2 : 1);
    if (VW > 1 && a.vec)
        madd_body<T, BX, BY, S, VW>(a);
    else
        madd_body<T, BX, BY, S, 1>(a);
}

}  // namespace pkk
