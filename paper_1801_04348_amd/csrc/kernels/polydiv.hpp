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

namespace pkk {

// The whole division in one launch (a program of this library, not one of
// the paper's): the K = n - M quotient coefficients first, then every
// remainder coefficient independently.  With top[j] the dividend coefficient
// at index n-1-j, step j of the division subtracts q_j b[M-d] from top[j+d]
// (1 <= d <= M), so q_k is top[k] after the steps before it -- a short
// sequential recurrence -- and the remainder is
//     r[x] = a[x] - sum_{0 <= j < K} q_j b[x - (K-1) + j]   (terms with a
//     b index below 0 vanish),
// K products per coefficient, no dependence between coefficients.
// Phase 1 runs in the first wavefront of every workgroup (redundantly, so no
// grid-wide synchronisation is needed): lane l keeps top[l + 64 r], r < R, in
// registers, the coefficient q_k is broadcast from its owner with a lane
// read, and b[M-1-i] is staged in LDS.  Phase 2: each workgroup stages the b
// window of its tile of S * B remainder coefficients and reads the quotient
// from LDS.  Needs K <= 64 * R <= 1024 and B >= 64.  LDS bytes:
// 4 * (2 * 1024 + S * B + 1024).  a[M .. n-1] are left for the host to clear.
constexpr int kPdMaxK = 1024;

__device__ __forceinline__ uint32_t barrett(uint64_t t, uint32_t P, uint64_t mu) {
    const uint64_t q = __umul64hi(t, mu);
    uint64_t r = t - q * P;
    if (r >= P) r -= P;
    return (uint32_t)r;
}

template <int B, int S, int R>
__device__ __forceinline__ void polydiv_fused(const PdArgs &g) {
    static_assert(B % 64 == 0 && R * 64 <= kPdMaxK, "fused division: whole wavefronts, K <= 1024");
    constexpr int TW = S * B;
    __shared__ uint32_t qs[kPdMaxK];
    __shared__ uint32_t bt[kPdMaxK];          // bt[i] = b[M-1-i]
    __shared__ uint32_t bw[TW + kPdMaxK];     // b window of a remainder tile
    const int M = g.M, n = g.n, K = n - M;
    const uint32_t P = g.P;
    const uint64_t mu = g.mu;
    const int t = threadIdx.x, lane = t & 63;
    const int nb = min(K, M);
    for (int i = t; i < nb; i += B) bt[i] = g.b[M - 1 - i];
    __syncthreads();
    if (t < 64) {
        uint32_t top[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int j = lane + 64 * r;
            top[r] = j < K ? g.a[n - 1 - j] : 0u;
        }
        for (int k = 0; k < K; ++k) {
            uint32_t mine = top[0];
#pragma unroll
            for (int r = 1; r < R; ++r)
                if (r == (k >> 6)) mine = top[r];
            const uint32_t q = (uint32_t)__builtin_amdgcn_readlane((int)mine, k & 63);
            if (lane == 0) qs[k] = q;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int d = lane + 64 * r - k;  // top[k + d] receives q b[M - d]
                if (d >= 1 && d <= nb && k + d < K) top[r] = submod(top[r], barrett((uint64_t)q * bt[d - 1], P, mu), P);
            }
        }
    }
    __syncthreads();
    const int tiles = (M + TW - 1) / TW;
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int x0 = tile * TW;
        for (int i = t; i < TW + K - 1; i += B) {
            const int p = x0 - (K - 1) + i;
            bw[i] = (p >= 0 && p < M) ? g.b[p] : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int xl = t + s * B, x = x0 + xl;
            if (x < M) {
                uint64_t acc = 0;
                for (int j = 0; j < K; ++j) acc += barrett((uint64_t)qs[j] * bw[xl + j], P, mu);
                g.a[x] = submod(g.a[x], barrett(acc, P, mu), P);
            }
        }
        __syncthreads();
    }
}

}  // namespace pkk
