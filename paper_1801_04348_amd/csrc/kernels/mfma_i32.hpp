// Wrapping int32 matrix product on the int8 matrix cores, for gfx950: the
// MFMA family's int32 programs (same contract as the float32 ones: C = [C +]
// A B, row-major, any M, N, K; the workgroup -> tile map and the 32 x 32
// block layout of mfma.hpp).
#pragma once

#include "mfma.hpp"

namespace pkk {

// ------------------------------------------------------------------ int32
// The wrapping int32 product on the int8 matrix cores (v_mfma_i32_32x32x32_i8:
// A 32x32 and B 32x32 of int8, C 32x32 of int32 per wavefront).  Every int32 x
// has four signed base-256 digits, x = sum_p d_p 256^p (mod 2^32) with d_p in
// [-128, 127]: the bytes of y = x + 0x80808080 (each byte v of y stands for
// v - 128), i.e. the bytes of y ^ 0x80808080 read as int8.  So
//   a b = sum over p + q <= 3 of 256^(p+q) d_p(a) d_q(b)   (mod 2^32):
// ten int8 products per pair of operand blocks, summed into four int32
// accumulators by p + q.  Each accumulator wraps modulo 2^32 as the result
// does, so combining them at the end, acc0 + 2^8 acc1 + 2^16 acc2 + 2^24
// acc3, gives the wrapped product exactly for every K.
// LDS, per stage: the four digit planes of the A tile (BM rows of BK bytes,
// k contiguous, rows BK + 16 bytes apart) and of the B tile stored by column
// (BN columns of BK bytes, k contiguous): 4 (BM + BN) (BK + 16) bytes.  With
// rows BK + 16 bytes apart (48 or 80) the sixteen 16-byte reads of a quarter
// wavefront, one per row, cover 64 distinct banks.
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

template <int BM, int BN, int BK, int STAGES> struct I32Lds {
    static constexpr int LD = BK + 16;                      // bytes per plane row
    static constexpr int A = 4 * BM * LD, B = 4 * BN * LD;  // bytes per stage
    static constexpr int bytes = STAGES * (A + B);
};

// The digit planes of four int32 values x[0..3] (consecutive k): byte e of
// plane word w[p] is digit p of x[e].
__device__ __forceinline__ void digit_planes(const i32x4 x, uint32_t w[4]) {
    uint32_t y[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) y[e] = ((uint32_t)x[e] + 0x80808080u) ^ 0x80808080u;
#pragma unroll
    for (int p = 0; p < 4; ++p)
        w[p] = ((y[0] >> (8 * p)) & 0xffu) | (((y[1] >> (8 * p)) & 0xffu) << 8) |
               (((y[2] >> (8 * p)) & 0xffu) << 16) | (((y[3] >> (8 * p)) & 0xffu) << 24);
}

// int32 tile (the whole K range).  A is read in 16-byte chunks of four k
// along its rows where `vec` (rows 16-byte aligned), else element by element;
// B element by element, four consecutive k of one column per work-item
// (lanes along the row: each load instruction reads 256 contiguous bytes), so
// B's leading dimension needs no alignment.  Rows of A past M and columns of B
// past N read the last row / column (their results are never stored);
// elements at k >= K are zeros (whose digits are zeros).
template <int BM, int BN, int BK, int WM, int WN, int STAGES>
__device__ __forceinline__ void mfma_i32_tile(const MmArgs &a, const int row0, const int col0, const bool vec,
                                              unsigned char *const As0, unsigned char *const Bs0) {
    constexpr int NT = 64 * WM * WN;
    constexpr int WTM = BM / WM, WTN = BN / WN;
    constexpr int TM = WTM / 32, TN = WTN / 32;
    using L = I32Lds<BM, BN, BK, STAGES>;
    constexpr int LD = L::LD;
    constexpr int AQ = BM * BK / 4 / NT;  // quads (four consecutive k) of A per work-item per step
    constexpr int BQ = BK * BN / 4 / NT;  // quads of B
    static_assert(TM >= 1 && TN >= 1 && WTM % 32 == 0 && WTN % 32 == 0, "wave tile must be 32x32 blocks");
    static_assert(AQ >= 1 && BQ >= 1 && (BM * BK / 4) % NT == 0 && (BK * BN / 4) % NT == 0, "tile loads");
    static_assert(BK % 32 == 0, "BK: whole MFMA steps in each half of the tile");

    const gptr<int32_t> __restrict__ A = (gptr<int32_t>)a.A;
    const gptr<int32_t> __restrict__ B = (gptr<int32_t>)a.B;
    const gmut<int32_t> __restrict__ C = (gmut<int32_t>)a.C;
    const int M = a.M, N = a.N, K = a.K;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int r = lane & 31, h = lane >> 5;
    const bool interior = (row0 + BM <= M) && (col0 + BN <= N);

    i32x16 acc[4][TM][TN];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[s][i][j][v] = 0;

    // each work-item's rows of A and columns of B, fixed for the tile (the
    // 64-bit address arithmetic done once, not per load and step)
    static_assert(NT % (BK / 4) == 0 && NT % BN == 0, "a work-item's A column and B column stay fixed");
    const int akq = 4 * (tid % (BK / 4));  // k offset of the work-item's A quads in a step
    gptr<int32_t> arow[AQ];
#pragma unroll
    for (int u = 0; u < AQ; ++u)
        arow[u] = A + (int64_t)min(row0 + (tid + u * NT) / (BK / 4), M - 1) * a.lda + akq;
    const int64_t ldb = a.ldb, ldb2 = 2 * ldb, ldb3 = 3 * ldb;
    // B: a work-item's BQ quads are consecutive in k (4 BQ of them from bk0),
    // so each digit plane takes one 4 BQ-byte LDS store per step: with one
    // four-byte store per quad, the 64 lanes' stores (one column each, rows
    // BK + 16 bytes apart) fell four to a bank
    const int bk0 = 4 * BQ * (tid / BN);
    gptr<int32_t> bcol[BQ];
#pragma unroll
    for (int u = 0; u < BQ; ++u) bcol[u] = B + (int64_t)(bk0 + 4 * u) * ldb + min(col0 + tid % BN, N - 1);

    i32x4 ra[AQ], rb[BQ];
    auto gload = [&](int k0) {
        const bool kfull = k0 + BK <= K;
#pragma unroll
        for (int u = 0; u < AQ; ++u) {
            const gptr<int32_t> q = arow[u] + k0;
            if (vec && kfull) {
                ra[u] = *reinterpret_cast<gptr<i32x4>>(q);
            } else {
                const int k = k0 + akq;
#pragma unroll
                for (int e = 0; e < 4; ++e) ra[u][e] = k + e < K ? q[e] : 0;
            }
        }
        const int64_t koff = (int64_t)k0 * ldb;
#pragma unroll
        for (int u = 0; u < BQ; ++u) {
            const gptr<int32_t> q[4] = {bcol[u] + koff, bcol[u] + koff + ldb, bcol[u] + koff + ldb2,
                                        bcol[u] + koff + ldb3};
            if (kfull) {
#pragma unroll
                for (int e = 0; e < 4; ++e) rb[u][e] = *q[e];
            } else {
                const int k = k0 + bk0 + 4 * u;
#pragma unroll
                for (int e = 0; e < 4; ++e) rb[u][e] = k + e < K ? *q[e] : 0;
            }
        }
    };
    auto sstore = [&](int st) {
        unsigned char *as = As0 + st * L::A;
        unsigned char *bs = Bs0 + st * L::B;
#pragma unroll
        for (int u = 0; u < AQ; ++u) {
            const int f = tid + u * NT;
            const int rr = f / (BK / 4), kq = f % (BK / 4);
            uint32_t w[4];
            digit_planes(ra[u], w);
#pragma unroll
            for (int p = 0; p < 4; ++p) *reinterpret_cast<uint32_t *>(as + p * BM * LD + rr * LD + 4 * kq) = w[p];
        }
        static_assert(BQ == 2 || BQ == 4, "a B run of 8 or 16 bytes per plane");
        typedef uint32_t brun __attribute__((ext_vector_type(BQ)));
        brun wb[4];
#pragma unroll
        for (int u = 0; u < BQ; ++u) {
            uint32_t w[4];
            digit_planes(rb[u], w);
#pragma unroll
            for (int p = 0; p < 4; ++p) wb[p][u] = w[p];
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) *reinterpret_cast<brun *>(bs + p * BN * LD + (tid % BN) * LD + bk0) = wb[p];
    };
    auto compute = [&](int st) {
        const unsigned char *as = As0 + st * L::A + (wm * WTM + r) * LD + h * (BK / 2);
        const unsigned char *bs = Bs0 + st * L::B + (wn * WTN + r) * LD + h * (BK / 2);
#pragma unroll
        for (int c = 0; c < BK / 2; c += 16) {
            i32x4 af[4][TM], bf[4][TN];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
#pragma unroll
                for (int i = 0; i < TM; ++i)
                    af[p][i] = *reinterpret_cast<const i32x4 *>(as + p * BM * LD + i * 32 * LD + c);
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    bf[p][j] = *reinterpret_cast<const i32x4 *>(bs + p * BN * LD + j * 32 * LD + c);
            }
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
#pragma unroll
                    for (int p = 0; p < 4; ++p)
#pragma unroll
                        for (int q = 0; p + q < 4; ++q)
                            acc[p + q][i][j] =
                                __builtin_amdgcn_mfma_i32_32x32x32_i8(af[p][i], bf[q][j], acc[p + q][i][j], 0, 0, 0);
        }
    };

    const int KT = (K + BK - 1) / BK;
    if (STAGES == 2) {
        if (KT > 0) {
            gload(0);
            sstore(0);
        }
        __syncthreads();
        for (int kt = 0; kt < KT; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < KT) gload((kt + 1) * BK);
            __builtin_amdgcn_sched_barrier(0);
            compute(cur);
            if (kt + 1 < KT) sstore(cur ^ 1);
            __syncthreads();
        }
    } else {
        if (KT > 0) gload(0);
        for (int kt = 0; kt < KT; ++kt) {
            __syncthreads();  // the previous step's LDS reads are done
            sstore(0);
            __syncthreads();
            if (kt + 1 < KT) gload((kt + 1) * BK);
            __builtin_amdgcn_sched_barrier(0);
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
                    const uint32_t x = (uint32_t)acc[0][i][j][v] + ((uint32_t)acc[1][i][j][v] << 8) +
                                       ((uint32_t)acc[2][i][j][v] << 16) + ((uint32_t)acc[3][i][j][v] << 24);
                    const gmut<int32_t> p = C + (int64_t)gr * a.ldc + gc;
                    *p = (int32_t)(a.accumulate ? (uint32_t)*p + x : x);
                }
            }
        }
}

// int32 programs: one form serves aligned and unaligned rows of A (WIDE
// false: element loads only), and none splits K.
template <int BM, int BN, int BK, int WM, int WN, int STAGES, bool WIDE = true>
__device__ __forceinline__ void mfma_i32(const MmArgs &a) {
    using L = I32Lds<BM, BN, BK, STAGES>;
    __shared__ __attribute__((aligned(16))) unsigned char As[STAGES * L::A];
    __shared__ __attribute__((aligned(16))) unsigned char Bs[STAGES * L::B];
    int tm, tn;
    tile_of(blockIdx.x, (a.M + BM - 1) / BM, (a.N + BN - 1) / BN, &tm, &tn);
    mfma_i32_tile<BM, BN, BK, WM, WN, STAGES>(a, tm * BM, tn * BN, WIDE && a.vec, As, Bs);
}

}  // namespace pkk
