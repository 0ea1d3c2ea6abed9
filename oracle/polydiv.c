/* Polynomial division modulo a prime -- TEST INFRASTRUCTURE ONLY.
 *
 * Section 5, Fig. 8 (polynomial division): a holds the N coefficients of a
 * polynomial over Z/PZ (a[i] multiplies x^i), b the M low coefficients of a
 * monic divisor of degree M (b(x) = x^M + b[M-1] x^(M-1) + ... + b[0]).
 * While the dividend's degree N - 1 is at least M, its leading coefficient
 * q = a[N-1] times x^(N-1-M) b(x) is subtracted:
 *     a[N-1-M+p] = (a[N-1-M+p] - q * b[p]) mod P,   0 <= p < M,
 * and N drops by one (a[N-1] is now zero).  On return a[0 .. min(N, M) - 1]
 * holds the remainder.  Residues are canonical, in [0, P); P >= 2 and
 * P < 2^31.  Plain loops in the figure's order.
 */
#include <stdint.h>

int oracle_polydiv_u32(uint32_t *a, int64_t N, const uint32_t *b, int64_t M, uint32_t P) {
    if (N < 0 || M < 1 || P < 2 || P >= 0x80000000u || (N > 0 && !a) || !b) return -1;
    for (int64_t i = 0; i < N; ++i)
        if (a[i] >= P) return -1;
    for (int64_t p = 0; p < M; ++p)
        if (b[p] >= P) return -1;
    for (int64_t n = N; n - 1 >= M; --n) {
        const uint64_t q = a[n - 1];
        for (int64_t p = 0; p < M; ++p) {
            const int64_t x = n - 1 - M + p;
            const uint64_t e = (q * b[p]) % P;
            a[x] = (uint32_t)((a[x] + (uint64_t)P - e) % P);
        }
        a[n - 1] = 0;
    }
    return 0;
}
