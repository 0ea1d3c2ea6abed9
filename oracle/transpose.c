/*
 * oracle/transpose.c -- TEST INFRASTRUCTURE ONLY.
 *
 * The plain definition of matrix transposition (Section 5.2, Fig. 7 and
 * Table 3): C (N x M) holds A (M x N) transposed, C[j][i] = A[i][j], for
 * 4-byte elements copied bit for bit.  Row-major with leading dimensions.
 */
#include <stdint.h>

int oracle_transpose_u32(const uint32_t *A, int64_t lda, uint32_t *C, int64_t ldc, int64_t M, int64_t N)
{
    if (M < 0 || N < 0 || (M > 0 && N > 0 && (lda < N || ldc < M))) return -1;
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j)
            C[j * ldc + i] = A[i * lda + j];
    return 0;
}
