"""Pins of the transposition oracle: a hand-worked case, involution, the
product identity (A B)^T = B^T A^T through the matmul oracle, and bit-exact
copying of arbitrary 4-byte patterns."""
import numpy as np

import oracle.matmul as om
import oracle.transpose as ot
from tests import inputs


def test_hand_worked():
    A = np.array([[1, 2, 3], [4, 5, 6]], dtype=np.int32)
    assert np.array_equal(ot.transpose(A), np.array([[1, 4], [2, 5], [3, 6]], dtype=np.int32))


def test_involution_and_shapes():
    A = inputs.full_range_i32((37, 91), seed=1).numpy()
    T = ot.transpose(A)
    assert T.shape == (91, 37)
    assert np.array_equal(ot.transpose(T), A)
    row = inputs.full_range_i32((1, 7), seed=2).numpy()
    assert ot.transpose(row).shape == (7, 1)


def test_product_identity():
    A = inputs.small_int_f32((13, 21), seed=3).numpy()
    B = inputs.small_int_f32((21, 8), seed=4).numpy()
    lhs = ot.transpose(om.matmul(A, B, "f32").astype(np.float32))
    rhs = om.matmul(ot.transpose(B), ot.transpose(A), "f32")
    assert np.array_equal(lhs.astype(np.float64), rhs)


def test_bit_patterns_preserved():
    bits = inputs.full_range_i32((16, 16), seed=5).numpy()
    f = bits.view(np.float32)          # includes NaN and denormal patterns
    assert np.array_equal(ot.transpose(f).view(np.int32), ot.transpose(bits))


def test_empty():
    assert ot.transpose(np.zeros((0, 5), np.float32)).shape == (5, 0)
