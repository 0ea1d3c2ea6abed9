"""Pins of the matrix-addition oracle: hand-worked values, commutativity,
the zero matrix, int32 wrap against Python integers, and float32 rounding
against numpy's float32 addition."""
import numpy as np

import oracle.madd as oa
from tests import inputs


def test_hand_worked():
    A = np.array([[1, 2, 3], [4, 5, 6]], dtype=np.int32)
    B = np.array([[10, 20, 30], [40, 50, 60]], dtype=np.int32)
    assert np.array_equal(oa.madd(A, B, "i32"), [[11, 22, 33], [44, 55, 66]])


def test_commutative_and_zero():
    A = inputs.full_range_i32((17, 33), seed=1).numpy()
    B = inputs.full_range_i32((17, 33), seed=2).numpy()
    assert np.array_equal(oa.madd(A, B, "i32"), oa.madd(B, A, "i32"))
    assert np.array_equal(oa.madd(A, np.zeros_like(A), "i32"), A)


def test_int32_wraps():
    A = inputs.full_range_i32((9, 11), seed=3).numpy()
    B = inputs.full_range_i32((9, 11), seed=4).numpy()
    C = oa.madd(A, B, "i32")
    for i in range(9):
        for j in range(11):
            s = (int(A[i, j]) + int(B[i, j])) % 2**32
            assert C[i, j] == (s - 2**32 if s >= 2**31 else s)


def test_float32_single_rounding():
    A = inputs.uniform_f32((20, 20), seed=5).numpy()
    B = inputs.uniform_f32((20, 20), seed=6).numpy()
    assert np.array_equal(oa.madd(A, B, "f32"), (A + B).astype(np.float32))
    # and agrees with the exact sum rounded once
    exact = A.astype(np.float64) + B.astype(np.float64)
    assert np.array_equal(oa.madd(A, B, "f32"), exact.astype(np.float32))
