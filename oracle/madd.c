/*
 * oracle/madd.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Matrix addition (Section 1, Fig. 1 and Fig. 2): C[i][j] = A[i][j] + B[i][j]
 * for an M x N row-major matrix with leading dimensions.  Fig. 1 writes it as
 * c = a + b and Fig. 2 as a = b + c (the array names are exchanged between the
 * two figures; the operation is the same).  int32 adds modulo 2^32 (unsigned
 * arithmetic); float32 adds in float32 (one rounding, exactly as the kernels).
 */
#include <stdint.h>

int oracle_madd_i32(const int32_t *A, int64_t lda, const int32_t *B, int64_t ldb, int32_t *C, int64_t ldc,
                    int64_t M, int64_t N)
{
    if (M < 0 || N < 0) return -1;
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j)
            C[i * ldc + j] = (int32_t)((uint32_t)A[i * lda + j] + (uint32_t)B[i * ldb + j]);
    return 0;
}

int oracle_madd_f32(const float *A, int64_t lda, const float *B, int64_t ldb, float *C, int64_t ldc, int64_t M,
                    int64_t N)
{
    if (M < 0 || N < 0) return -1;
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j)
            C[i * ldc + j] = A[i * lda + j] + B[i * ldb + j];
    return 0;
}
