// Parametric matrix addition (Section 1, Fig. 1 and Fig. 2), for gfx950.
//
// C = A + B for M x N row-major matrices with leading dimensions.  A
// workgroup of BX x BY work-items owns BY rows and BX * S columns; work-item
// (ty, tx) adds the S elements of row ty at columns tx + w * BX, w < S, so the
// lanes of a wavefront touch consecutive addresses (Fig. 2's K1 adds the two
// elements j and j + N/2 of a row; here the S elements of a thread are BX
// apart, which keeps every access coalesced for any S).  After granularity
// reduction (Fig. 2's K2) S = 1.  int32 adds modulo 2^32; float32 adds with
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
};

template <typename T> struct AddOp;
template <> struct AddOp<float> {
    static __device__ __forceinline__ float add(float a, float b) { return a + b; }
};
template <> struct AddOp<int32_t> {
    static __device__ __forceinline__ int32_t add(int32_t a, int32_t b) { return (int32_t)((uint32_t)a + (uint32_t)b); }
};

template <typename T, int BX, int BY, int S>
__device__ __forceinline__ void madd(const MaArgs &a) {
    constexpr int TN = BX * S;
    const T *__restrict__ A = static_cast<const T *>(a.A);
    const T *__restrict__ B = static_cast<const T *>(a.B);
    T *__restrict__ C = static_cast<T *>(a.C);
    const int M = a.M, N = a.N;
    const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
    const int tiles_n = (N + TN - 1) / TN;
    const int64_t tiles = (int64_t)((M + BY - 1) / BY) * tiles_n;
    for (int64_t b = blockIdx.x; b < tiles; b += gridDim.x) {
        const int row = (int)(b / tiles_n) * BY + ty;
        const int col0 = (int)(b % tiles_n) * TN + tx;
        if (row >= M) continue;
        T va[S], vb[S];
#pragma unroll
        for (int w = 0; w < S; ++w) {
            const int col = col0 + w * BX;
            va[w] = col < N ? A[(int64_t)row * a.lda + col] : T(0);
            vb[w] = col < N ? B[(int64_t)row * a.ldb + col] : T(0);
        }
#pragma unroll
        for (int w = 0; w < S; ++w) {
            const int col = col0 + w * BX;
            if (col < N) C[(int64_t)row * a.ldc + col] = AddOp<T>::add(va[w], vb[w]);
        }
    }
}

}  // namespace pkk
