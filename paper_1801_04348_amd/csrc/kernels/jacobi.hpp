// Parametric 1D Jacobi step (Section 5, Fig. 6, Table 2), for gfx950.
//
// One time step of the paper's three-point stencil over the two halves of a
// length-2N array: with `in` one half and `out` the other, for every interior
// point p + 1, p < n = N - 2,
//     out[p + 1] = (in[p] + in[p + 1] + in[p + 2]) / 3,
// evaluated left to right: int32 sums wrap modulo 2^32 and the quotient
// truncates toward zero (C semantics); float32 rounds after each addition and
// after the (correctly rounded) division.  The end points out[0], out[N - 1]
// are never written.
//
// A workgroup of B work-items owns S * B consecutive outputs; work-item j
// computes outputs j + k * B, k < S (the paper's p = j + (i s + k) B), so the
// lanes of a wavefront always touch consecutive addresses.
// jacobi_tiled (the paper's cache(a) programs): the S * B + 2 inputs of the
//   tile are staged in LDS with coalesced loads, then each output reads its
//   three neighbours from LDS.  LDS bytes: 4 * (S * B + 2).  After granularity
//   reduction S = 1.
// jacobi_direct (no caching, decision (4b)): each output reads its three
//   neighbours from global memory (the cache hierarchy absorbs the reuse).
// Pure streaming: HBM-bound, 8 bytes per point and step at best.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pkk {

struct JaArgs {
    const void *in;
    void *out;
    int32_t n;  // interior points: N - 2
};

template <typename T> struct Avg3;
template <> struct Avg3<float> {
    static __device__ __forceinline__ float f(float a, float b, float c) { return ((a + b) + c) / 3.0f; }
};
template <> struct Avg3<int32_t> {
    static __device__ __forceinline__ int32_t f(int32_t a, int32_t b, int32_t c) {
        return (int32_t)((uint32_t)a + (uint32_t)b + (uint32_t)c) / 3;
    }
};

template <typename T, int B, int S>
__device__ __forceinline__ void jacobi_tiled(const JaArgs &a) {
    constexpr int TW = S * B;
    __shared__ T buf[TW + 2];
    const T *__restrict__ in = static_cast<const T *>(a.in);
    T *__restrict__ out = static_cast<T *>(a.out);
    const int n = a.n, t = threadIdx.x;
    const int tiles = (n + TW - 1) / TW;
    for (int b = blockIdx.x; b < tiles; b += gridDim.x) {
        const int p0 = b * TW;
        const int have = min(TW, n - p0) + 2;  // inputs this tile reads
#pragma unroll
        for (int k = 0; k <= S; ++k) {
            const int e = t + k * B;
            if (e < have) buf[e] = in[p0 + e];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const int q = t + k * B;
            if (q < have - 2) out[p0 + q + 1] = Avg3<T>::f(buf[q], buf[q + 1], buf[q + 2]);
        }
        __syncthreads();
    }
}

template <typename T, int B, int S>
__device__ __forceinline__ void jacobi_direct(const JaArgs &a) {
    constexpr int TW = S * B;
    const T *__restrict__ in = static_cast<const T *>(a.in);
    T *__restrict__ out = static_cast<T *>(a.out);
    const int n = a.n, t = threadIdx.x;
    const int tiles = (n + TW - 1) / TW;
    for (int b = blockIdx.x; b < tiles; b += gridDim.x) {
        const int p0 = b * TW;
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const int p = p0 + t + k * B;
            if (p < n) out[p + 1] = Avg3<T>::f(in[p], in[p + 1], in[p + 2]);
        }
    }
}

}  // namespace pkk
