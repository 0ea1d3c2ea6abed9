/*
 * oracle/matmul.c -- TEST INFRASTRUCTURE ONLY.
 *
 * The plain, slow CPU definition of the product that the parametric kernels
 * compute.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark load this file's library; the product never links it, and it
 * shares no header, helper or constant with the HIP tree.
 *
 * What is computed (the blocked product of Section 2, Fig. 3, whose innermost
 * statement adds a[p][k] * b[k][q] into c[p][q]; generalised from square
 * order n to rectangular row-major operands with leading dimensions):
 *
 *     C[i][j] = (accumulate ? Cin[i][j] : 0) + sum_{k = 0}^{K-1} A[i][k] * B[k][j]
 *
 * The kernel of Fig. 4 first loads c into registers and writes it back after
 * the K loop, i.e. it accumulates into C; ``accumulate = 1`` reproduces that,
 * ``accumulate = 0`` overwrites.
 *
 * Arithmetic:
 *   - float32 and bfloat16 inputs are converted exactly to double and the sum
 *     is taken in double, in the order k = 0, 1, ..., K-1 (Cin first);
 *   - int32 inputs use unsigned 32-bit arithmetic, i.e. every product and sum
 *     is reduced modulo 2^32 and the result reinterpreted as int32 (signed
 *     overflow is undefined behaviour in C, unsigned wrap is not).
 *
 * Loop order is i-k-j over a row buffer; OpenMP splits the rows i.  Neither
 * changes the per-element order of the sum over k.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_BAD_ARG -1

static int bad_shape(int64_t M, int64_t N, int64_t K, int64_t lda, int64_t ldb, int64_t ldc)
{
    if (M < 0 || N < 0 || K < 0) return 1;
    if (M > 0 && K > 0 && lda < K) return 1;
    if (K > 0 && N > 0 && ldb < N) return 1;
    if (M > 0 && N > 0 && ldc < N) return 1;
    return 0;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* exact value of a bfloat16 bit pattern: the high half of a float32 */
static double bf16_value(uint16_t bits)
{
    uint32_t w = ((uint32_t)bits) << 16;
    float f;
    memcpy(&f, &w, sizeof f);
    return (double)f;
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* float32 inputs; C and Cin are double, row-major with leading dimension ldc */
int oracle_matmul_f32(const float *A, int64_t lda, const float *B, int64_t ldb,
                      const double *Cin, double *C, int64_t ldc,
                      int64_t M, int64_t N, int64_t K, int accumulate, int nthreads)
{
    if (bad_shape(M, N, K, lda, ldb, ldc)) return ORACLE_BAD_ARG;
    if (M == 0 || N == 0) return ORACLE_OK;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        double *row = C + i * ldc;
        for (int64_t j = 0; j < N; ++j)
            row[j] = accumulate ? Cin[i * ldc + j] : 0.0;
        for (int64_t k = 0; k < K; ++k) {
            const double a = (double)A[i * lda + k];
            const float *brow = B + k * ldb;
            for (int64_t j = 0; j < N; ++j)
                row[j] += a * (double)brow[j];
        }
    }
    return ORACLE_OK;
}

/* bfloat16 inputs given as raw bit patterns; exact values, double sum */
int oracle_matmul_bf16(const uint16_t *A, int64_t lda, const uint16_t *B, int64_t ldb,
                       const double *Cin, double *C, int64_t ldc,
                       int64_t M, int64_t N, int64_t K, int accumulate, int nthreads)
{
    if (bad_shape(M, N, K, lda, ldb, ldc)) return ORACLE_BAD_ARG;
    if (M == 0 || N == 0) return ORACLE_OK;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        double *row = C + i * ldc;
        for (int64_t j = 0; j < N; ++j)
            row[j] = accumulate ? Cin[i * ldc + j] : 0.0;
        for (int64_t k = 0; k < K; ++k) {
            const double a = bf16_value(A[i * lda + k]);
            const uint16_t *brow = B + k * ldb;
            for (int64_t j = 0; j < N; ++j)
                row[j] += a * bf16_value(brow[j]);
        }
    }
    return ORACLE_OK;
}

/* int32 inputs, arithmetic modulo 2^32 */
int oracle_matmul_i32(const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb,
                      const int32_t *Cin, int32_t *C, int64_t ldc,
                      int64_t M, int64_t N, int64_t K, int accumulate, int nthreads)
{
    if (bad_shape(M, N, K, lda, ldb, ldc)) return ORACLE_BAD_ARG;
    if (M == 0 || N == 0) return ORACLE_OK;
    set_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i) {
        uint32_t *row = (uint32_t *)malloc((size_t)N * sizeof(uint32_t));
        for (int64_t j = 0; j < N; ++j)
            row[j] = accumulate ? (uint32_t)Cin[i * ldc + j] : 0u;
        for (int64_t k = 0; k < K; ++k) {
            const uint32_t a = (uint32_t)A[i * lda + k];
            const int32_t *brow = B + k * ldb;
            for (int64_t j = 0; j < N; ++j)
                row[j] += a * (uint32_t)brow[j];
        }
        for (int64_t j = 0; j < N; ++j)
            C[i * ldc + j] = (int32_t)row[j];
        free(row);
    }
    return ORACLE_OK;
}

/* One element computed on its own: used to check sampled outputs of the full
 * sizes without computing the whole product. */
double oracle_dot_f32(const float *A, int64_t lda, const float *B, int64_t ldb,
                      int64_t i, int64_t j, int64_t K)
{
    double s = 0.0;
    for (int64_t k = 0; k < K; ++k)
        s += (double)A[i * lda + k] * (double)B[k * ldb + j];
    return s;
}

double oracle_dot_bf16(const uint16_t *A, int64_t lda, const uint16_t *B, int64_t ldb,
                       int64_t i, int64_t j, int64_t K)
{
    double s = 0.0;
    for (int64_t k = 0; k < K; ++k)
        s += bf16_value(A[i * lda + k]) * bf16_value(B[k * ldb + j]);
    return s;
}

int32_t oracle_dot_i32(const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb,
                       int64_t i, int64_t j, int64_t K)
{
    uint32_t s = 0u;
    for (int64_t k = 0; k < K; ++k)
        s += (uint32_t)A[i * lda + k] * (uint32_t)B[k * ldb + j];
    return (int32_t)s;
}
