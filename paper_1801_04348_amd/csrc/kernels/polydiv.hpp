// Parametric polynomial division modulo a prime (Section 5, Fig. 8, Table 4),
// for gfx950.
//
// a holds the n coefficients of the dividend (a[i] multiplies x^i), b the M
// low coefficients of a monic divisor of degree M; residues in [0, P),
// P < 2^31.  One step (the body of the figure's while loop, one launch) with
// q = a[n-1]:
//     a[n-1-M+p] = (a[n-1-M+p] - q b[p]) mod P,   0 <= p < M,
// which eliminates the leading coefficient; its slot a[n-1] is not read
// again, and the host clears a[M .. N-1] once after the last step (clearing
// it inside a step would race with workgroups still reading q).  A workgroup
// of B work-items owns S * B consecutive p; work-item j takes p = j + k * B,
// k < S, so lanes touch consecutive addresses.
// polydiv_step_tiled (the figure's cache(a, b) programs): the tile's a and b
//   values and q are staged in LDS with coalesced loads first.  LDS bytes:
//   4 * (2 * S * B + 1).  After granularity reduction S = 1.
// polydiv_step_direct (no caching, decision (4b)): operands straight from
//   global memory; q is one address every lane reads (a cache broadcast).
// Products are reduced by Barrett's method with mu = floor(2^64 / P): for
// x < P^2 < 2^62 the estimate floor(x mu / 2^64) is the quotient or one less.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pkk {

struct PdArgs {
    uint32_t *a;
    const uint32_t *b;
    int32_t M;
    int32_t n;      // current number of dividend coefficients, n - 1 >= M
    uint32_t P;
    uint64_t mu;    // floor(2^64 / P)
};

__device__ __forceinline__ uint32_t mulmod(uint32_t x, uint32_t y, uint32_t P, uint64_t mu) {
    const uint64_t t = (uint64_t)x * y;
    const uint64_t q = __umul64hi(t, mu);
    uint64_t r = t - q * P;
    if (r >= P) r -= P;
    return (uint32_t)r;
}

__device__ __forceinline__ uint32_t submod(uint32_t x, uint32_t y, uint32_t P) {
    return x >= y ? x - y : x + (P - y);
}

template <int B, int S>
__device__ __forceinline__ void polydiv_step_tiled(const PdArgs &g) {
    constexpr int TW = S * B;
    __shared__ uint32_t sa[TW], sb[TW], sq;
    const int M = g.M, t = threadIdx.x;
    const int base = g.n - 1 - M;  // a index of p = 0
    const int tiles = (M + TW - 1) / TW;
    if (t == 0) sq = g.a[g.n - 1];
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int p0 = tile * TW;
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const int p = p0 + t + k * B;
            if (p < M) {
                sa[t + k * B] = g.a[base + p];
                sb[t + k * B] = g.b[p];
            }
        }
        __syncthreads();
        const uint32_t q = sq;
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const int p = p0 + t + k * B;
            if (p < M) g.a[base + p] = submod(sa[t + k * B], mulmod(q, sb[t + k * B], g.P, g.mu), g.P);
        }
        __syncthreads();
    }
}

template <int B, int S>
__device__ __forceinline__ void polydiv_step_direct(const PdArgs &g) {
    constexpr int TW = S * B;
    const int M = g.M, t = threadIdx.x;
    const int base = g.n - 1 - M;
    const int tiles = (M + TW - 1) / TW;
    const uint32_t q = g.a[g.n - 1];
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int p0 = tile * TW;
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const int p = p0 + t + k * B;
            if (p < M) g.a[base + p] = submod(g.a[base + p], mulmod(q, g.b[p], g.P, g.mu), g.P);
        }
    }
}

}  // namespace pkk
