"""Pins of the 1D Jacobi oracle (Section 5, Fig. 6) against facts fixed by
the mathematics: trinomial coefficients of a spike, fixed points, hand-worked
truncation and wrap-around, the error bound of float32, untouched ends."""
import math

import numpy as np
import pytest

import oracle.jacobi as oj
from tests import inputs


def both(first):
    first = np.asarray(first)
    return np.concatenate([first, first])


def test_spike_spreads_as_trinomial_coefficients():
    # averaging three neighbours T times spreads a spike of 3^T as the
    # coefficients of (1 + x + x^2)^T; divisions are exact, ends far away
    T, N, c = 6, 41, 20
    a = np.zeros(N, dtype=np.int64)
    a[c] = 3 ** T
    out = oj.result_half(oj.jacobi1d(both(a), T, "i32"), T)
    coeff = np.array([1])
    for _ in range(T):
        coeff = np.convolve(coeff, [1, 1, 1])
    want = np.zeros(N, dtype=np.int64)
    want[c - T:c + T + 1] = coeff
    assert np.array_equal(out, want)
    assert coeff.sum() == 3 ** T


def test_linear_profile_is_a_fixed_point():
    N = 37
    for dtype in ("i32", "f32"):
        lin = np.arange(N) * 5 - 40
        out = oj.jacobi1d(both(lin), 5, dtype)
        assert np.array_equal(out[:N], lin) and np.array_equal(out[N:], lin)


def test_hand_worked_truncation_toward_zero():
    # (-1 + 0 + 0) / 3 truncates to 0 (floor would give -1); (-4 + 0 + 0) / 3 = -1
    a = both([0, -1, 0, 0, -4, 0, 0])
    out = oj.jacobi1d(a, 1, "i32")
    assert list(out[7:]) == [0, 0, 0, -1, -1, -1, 0]
    assert list(out[:7]) == [0, -1, 0, 0, -4, 0, 0]     # first copy untouched by an even step


def test_hand_worked_wraparound():
    # 3 * (2^31 - 1) = 6442450941 wraps to 2147483645 (mod 2^32, signed), / 3 -> 715827881
    m = 2 ** 31 - 1
    out = oj.jacobi1d(both([m, m, m]), 1, "i32")
    assert out[4] == 715827881
    # -2^31 * 3 wraps to -2^31, / 3 -> -715827882 (truncated from -715827882.67)
    n = -2 ** 31
    out = oj.jacobi1d(both([n, n, n]), 1, "i32")
    assert out[4] == -715827882


def test_float32_within_rounding_bound_of_exact_average():
    N, T = 257, 1
    a = inputs.uniform_f32((2 * N,), seed=3).numpy()
    out = oj.jacobi1d(a, T, "f32")
    x = a[:N].astype(np.float64)
    exact = (x[:-2] + x[1:-1] + x[2:]) / 3
    bound = 3 * 2.0 ** -24 * (np.abs(x[:-2]) + np.abs(x[1:-1]) + np.abs(x[2:])) / 3 * 1.01
    assert np.all(np.abs(out[N + 1:2 * N - 1] - exact) <= bound + 1e-45)


def test_steps_alternate_and_ends_stay():
    N = 11
    a = inputs.small_int_i32((2 * N,), seed=5).numpy()
    for T in range(0, 5):
        out = oj.jacobi1d(a, T, "i32")
        for i in (0, N - 1, N, 2 * N - 1):
            assert out[i] == a[i]
        if T >= 1:
            # step 1 wrote the second copy from the first: one further step from the
            # oracle's own result reproduces T steps (composition)
            prev = oj.jacobi1d(a, T - 1, "i32")
            nxt = prev.copy()
            src, dst = (prev[N:], nxt[:N]) if (T - 1) % 2 else (prev[:N], nxt[N:])
            s = (src[:-2].astype(np.int64) + src[1:-1] + src[2:])
            dst[1:-1] = np.trunc(s / 3).astype(np.int64)   # small values: no wrap
            assert np.array_equal(out, nxt)


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oj.jacobi1d(np.zeros(3), 1, "i32")
    with pytest.raises(ValueError):
        oj.jacobi1d(np.zeros(2), 1, "i32")   # N = 1
