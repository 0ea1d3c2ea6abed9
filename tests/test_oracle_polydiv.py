"""Pins of the polynomial-division oracle (Section 5, Fig. 8) against facts
fixed by the mathematics: a hand-worked quotient, q*b + r rebuilt with
Python integers, the remainder theorem, a GF(2) reduction."""
import numpy as np
import pytest

import oracle.polydiv as opd

P31 = 2147483647   # 2^31 - 1, prime


def test_hand_worked():
    # (x^3 + 2x + 1) = x (x^2 + 1) + (x + 1) over Z/7
    out = opd.polydiv([1, 2, 0, 1], [1, 0], 7)
    assert list(out) == [1, 1, 0, 0]


def test_gf2_reduction():
    # x^5 mod (x^4 + x + 1) = x^2 + x over GF(2)
    out = opd.polydiv([0, 0, 0, 0, 0, 1], [1, 1, 0, 0], 2)
    assert list(out[:4]) == [0, 1, 1, 0] and not out[4:].any()


def _mul_mod(u, v, P):
    out = [0] * (len(u) + len(v) - 1)
    for i, x in enumerate(u):
        for j, y in enumerate(v):
            out[i + j] = (out[i + j] + x * y) % P
    return out


@pytest.mark.parametrize("P,M,K", [(P31, 7, 5), (65521, 12, 30), (3, 4, 9), (P31, 1, 3)])
def test_rebuilds_quotient_times_divisor_plus_remainder(P, M, K):
    rng = np.random.default_rng(P % 1000 + M + K)
    q = [int(x) for x in rng.integers(0, P, K)]
    low = [int(x) for x in rng.integers(0, P, M)]
    r = [int(x) for x in rng.integers(0, P, M)]
    b = low + [1]                                  # monic of degree M
    a = _mul_mod(q, b, P)
    a = [(a[i] + (r[i] if i < M else 0)) % P for i in range(len(a))]
    out = opd.polydiv(a, low, P)
    assert [int(x) for x in out[:M]] == r
    assert not out[M:].any()


def test_remainder_theorem():
    # a mod (x - c) = a(c) mod P
    P = 1000003
    rng = np.random.default_rng(7)
    a = [int(x) for x in rng.integers(0, P, 50)]
    for c in (0, 1, 5, P - 1, 123457):
        val = 0
        for coef in reversed(a):
            val = (val * c + coef) % P
        out = opd.polydiv(a, [(P - c) % P], P)
        assert int(out[0]) == val and not out[1:].any()


def test_short_dividend_unchanged_and_errors():
    out = opd.polydiv([3, 4], [1, 2, 5], 7)
    assert list(out) == [3, 4]
    with pytest.raises(ValueError):
        opd.polydiv([9], [1], 7)          # residue >= P
    with pytest.raises(ValueError):
        opd.polydiv([1], [], 7)           # M = 0
    with pytest.raises(ValueError):
        opd.polydiv([1], [1], 1)          # P < 2
