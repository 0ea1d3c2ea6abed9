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
        if (have == TW + 2) {
            // a full tile: the S loads of a work-item go out together (a
            // guard per load makes each wait for the one before)
            T v[S];
#pragma unroll
            for (int k = 0; k < S; ++k) v[k] = in[p0 + t + k * B];
            if (t < 2) buf[TW + t] = in[p0 + TW + t];
#pragma unroll
            for (int k = 0; k < S; ++k) buf[t + k * B] = v[k];
        } else {
#pragma unroll
            for (int k = 0; k <= S; ++k) {
                const int e = t + k * B;
                if (e < have) buf[e] = in[p0 + e];
            }
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
        if (p0 + TW <= n) {  // a full tile: loads out together
            T x[S], y[S], z[S];
#pragma unroll
            for (int k = 0; k < S; ++k) {
                const int p = p0 + t + k * B;
                x[k] = in[p];
                y[k] = in[p + 1];
                z[k] = in[p + 2];
            }
#pragma unroll
            for (int k = 0; k < S; ++k) out[p0 + t + k * B + 1] = Avg3<T>::f(x[k], y[k], z[k]);
            continue;
        }
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const int p = p0 + t + k * B;
            if (p < n) out[p + 1] = Avg3<T>::f(in[p], in[p + 1], in[p + 2]);
        }
    }
}

}  // namespace pkk

namespace pkk {

// Several time steps in one launch (a program of this library, not one of
// the paper's): each workgroup stages its tile of S * B interior points with
// a halo of k points on each side in LDS, advances the window k steps there
// (the valid part shrinking by one point per side per step), and writes the
// tile's points after k steps to the other half.  The end points are never
// written, and each step reads those of the half it reads: the input half's
// for odd steps of the launch, the output half's for even ones.  The arithmetic of every point and step is the
// per-step kernels', so results are bit-identical; the halo is recomputed by
// neighbouring workgroups instead of exchanged.  k is odd, 1 <= k <
// kJaMaxSteps: after an odd number of steps the state belongs in the other
// half, exactly where the per-step schedule would have put it.
// LDS bytes: 2 * 4 * (S * B + 2 * kJaMaxSteps).
constexpr int kJaMaxSteps = 16;

struct JfArgs {
    const void *in;
    void *out;
    int32_t N;  // points per half
    int32_t k;  // steps this launch
};

template <typename T, int B, int S>
__device__ __forceinline__ void jacobi_fused(const JfArgs &a) {
    constexpr int TW = S * B, LW = TW + 2 * kJaMaxSteps;
    __shared__ T buf[2][LW];
    const T *__restrict__ in = static_cast<const T *>(a.in);
    T *__restrict__ out = static_cast<T *>(a.out);
    const int N = a.N, k = a.k, t = threadIdx.x;
    const int n = N - 2, L = TW + 2 * k;
    const T in0 = in[0], inN = in[N - 1], out0 = out[0], outN = out[N - 1];
    const int tiles = (n + TW - 1) / TW;
    for (int b = blockIdx.x; b < tiles; b += gridDim.x) {
        const int g0 = 1 + b * TW;  // first interior point of the tile
        const int w0 = g0 - k;      // window start (may lie before the vector)
        if (w0 >= 0 && w0 + L <= N) {
            // the window lies inside the vector: the first S chunks (i < TW <=
            // L) load together, then the 2k points left
            T v[S];
#pragma unroll
            for (int c = 0; c < S; ++c) v[c] = in[w0 + t + c * B];
#pragma unroll
            for (int c = 0; c < S; ++c) buf[0][t + c * B] = v[c];
            for (int i = TW + t; i < L; i += B) buf[0][i] = in[w0 + i];
        } else {
            for (int i = t; i < L; i += B) {
                const int g = w0 + i;
                buf[0][i] = (g >= 0 && g < N) ? in[g] : T(0);
            }
        }
        __syncthreads();
        for (int j = 1; j <= k; ++j) {
            const T *src = buf[(j - 1) & 1];
            T *dst = buf[j & 1];
            for (int i = j + t; i < L - j; i += B) {
                const int g = w0 + i;
                if (g == 0)
                    dst[i] = (j & 1) ? out0 : in0;  // the ends of the half step j wrote
                else if (g == N - 1)
                    dst[i] = (j & 1) ? outN : inN;
                else if (g < 0 || g >= N)
                    dst[i] = src[i];  // outside the vector: never read by a valid point
                else
                    dst[i] = Avg3<T>::f(src[i - 1], src[i], src[i + 1]);
            }
            __syncthreads();
        }
        const T *res = buf[k & 1];
        for (int o = t; o < TW; o += B) {
            const int g = g0 + o;
            if (g < N - 1) out[g] = res[k + o];
        }
        __syncthreads();
    }
}

}  // namespace pkk
