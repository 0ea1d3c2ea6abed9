/* 1D Jacobi oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Section 5, Fig. 6 (the source program of the 1D Jacobi example): an array
 * of 2N elements holds two copies of a length-N vector.  Step t, for every
 * interior index p + 1 with 0 <= p < N - 2:
 *   t even: second copy  a[N + p + 1] = (a[p] + a[p + 1] + a[p + 2]) / 3
 *   t odd:  first copy   a[p + 1]     = (a[N + p] + a[N + p + 1] + a[N + p + 2]) / 3
 * Elements 0, N - 1, N and 2N - 1 are never written.  int32: the sum wraps
 * modulo 2^32 (the paper's int type, with overflow defined as wrapping) and
 * the division truncates toward zero; float32: one rounding per addition,
 * left to right, and one for the division.  Plain loops, in the paper's
 * order of steps.
 */
#include <stdint.h>

int oracle_jacobi1d_i32(int32_t *a, int64_t N, int64_t T) {
    if (N < 2 || T < 0 || (!a && N > 0)) return -1;
    for (int64_t t = 0; t < T; ++t) {
        const int32_t *src = (t % 2) ? a + N : a;
        int32_t *dst = (t % 2) ? a : a + N;
        for (int64_t p = 0; p < N - 2; ++p) {
            uint32_t s = (uint32_t)src[p] + (uint32_t)src[p + 1] + (uint32_t)src[p + 2];
            dst[p + 1] = (int32_t)s / 3;
        }
    }
    return 0;
}

int oracle_jacobi1d_f32(float *a, int64_t N, int64_t T) {
    if (N < 2 || T < 0 || (!a && N > 0)) return -1;
    for (int64_t t = 0; t < T; ++t) {
        const float *src = (t % 2) ? a + N : a;
        float *dst = (t % 2) ? a : a + N;
        for (int64_t p = 0; p < N - 2; ++p) {
            float s = src[p] + src[p + 1];
            s = s + src[p + 2];
            dst[p + 1] = s / 3.0f;
        }
    }
    return 0;
}
