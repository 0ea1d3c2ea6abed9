"""Pins of the matmul oracle against values fixed by mathematics, not by itself.

The oracle follows the blocked product of Section 2 (Fig. 3): C[i][j] sums
A[i][k] * B[k][j] over k (plus C_in when accumulating, as the kernel of Fig. 4
does).  Each test below would fail for a plausible slip in it: a transposed
operand, a dropped or doubled term, a wrong stride, a lost accumulate input, a
signed-overflow shortcut for int32, a wrong bfloat16 decode.
"""
import numpy as np
import pytest

import oracle.matmul as om
from tests import inputs


def test_hand_computed_rectangular():
    # 2x3 by 3x2, worked by hand: [[1,2,3],[4,5,6]] @ [[7,8],[9,10],[11,12]]
    A = np.array([[1, 2, 3], [4, 5, 6]], dtype=np.float32)
    B = np.array([[7, 8], [9, 10], [11, 12]], dtype=np.float32)
    want = np.array([[58, 64], [139, 154]], dtype=np.float64)
    assert np.array_equal(om.matmul(A, B, "f32"), want)
    # the transpose product differs, so a swapped operand would be caught
    assert not np.array_equal(om.matmul(B.T.copy(), A.T.copy(), "f32"), want)


@pytest.mark.parametrize("M,N,K", [(m, n, k) for m in (1, 2, 5, 9) for n in (1, 3, 8) for k in (1, 4, 7, 9)])
def test_brute_force_tiny_vs_numpy_float64(M, N, K):
    A = inputs.uniform_f32((M, K), seed=M * 100 + N * 10 + K)
    B = inputs.uniform_f32((K, N), seed=M * 100 + N * 10 + K + 7)
    want = A.numpy().astype(np.float64) @ B.numpy().astype(np.float64)
    got = om.matmul(A, B, "f32")
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12)


def test_identity_returns_b_exactly():
    B = inputs.uniform_f32((33, 17), seed=3)
    I = np.eye(33, dtype=np.float32)
    assert np.array_equal(om.matmul(I, B, "f32"), B.numpy().astype(np.float64))


def test_one_hot_row_selects_row():
    B = inputs.uniform_f32((10, 6), seed=4)
    A = np.zeros((3, 10), dtype=np.float32)
    A[0, 7] = 1.0
    A[2, 0] = 1.0
    C = om.matmul(A, B, "f32")
    assert np.array_equal(C[0], B.numpy()[7].astype(np.float64))
    assert np.all(C[1] == 0.0)
    assert np.array_equal(C[2], B.numpy()[0].astype(np.float64))


def test_accumulate_adds_cin():
    A = inputs.uniform_f32((4, 5), seed=5)
    B = inputs.uniform_f32((5, 3), seed=6)
    Cin = np.arange(12, dtype=np.float64).reshape(4, 3)
    got = om.matmul(A, B, "f32", Cin=Cin)
    assert np.allclose(got - Cin, A.numpy().astype(np.float64) @ B.numpy().astype(np.float64), atol=1e-14)


def test_k_zero_gives_zero_or_cin():
    A = np.zeros((3, 0), dtype=np.float32)
    B = np.zeros((0, 4), dtype=np.float32)
    assert np.all(om.matmul(A, B, "f32") == 0.0)
    Cin = np.full((3, 4), 2.5)
    assert np.all(om.matmul(A, B, "f32", Cin=Cin) == 2.5)


def test_small_integer_sums_are_exact():
    # integer inputs with |a|,|b| <= 8: every partial sum is an integer, so
    # the double result equals exact integer arithmetic (Python ints)
    A = inputs.small_int_i32((6, 50), seed=7)
    B = inputs.small_int_i32((50, 5), seed=8)
    got = om.matmul(A.float(), B.float(), "f32")
    a, b = A.tolist(), B.tolist()
    want = [[sum(a[i][k] * b[k][j] for k in range(50)) for j in range(5)] for i in range(6)]
    assert np.array_equal(got, np.array(want, dtype=np.float64))


def test_int32_wraps_modulo_2_32():
    A = inputs.full_range_i32((5, 13), seed=9)
    B = inputs.full_range_i32((13, 4), seed=10)
    got = om.matmul(A, B, "i32")
    a, b = A.tolist(), B.tolist()
    for i in range(5):
        for j in range(4):
            s = sum(a[i][k] * b[k][j] for k in range(13)) % 2**32
            if s >= 2**31:
                s -= 2**32
            assert got[i, j] == s


def test_int32_edge_values():
    # 2^30 * 2 + 2^30 * 1 = 3 * 2^30 exceeds 2^31 - 1 and wraps to -2^30
    A = np.array([[2**30, 2**30]], dtype=np.int32)
    B = np.array([[2], [1]], dtype=np.int32)
    assert om.matmul(A, B, "i32")[0, 0] == -(2**30)
    # (2^31 - 1) * 2 + (-2^31) * 1 = 2^31 - 2: large terms, no net wrap
    A2 = np.array([[2**31 - 1, -(2**31)]], dtype=np.int32)
    assert om.matmul(A2, B, "i32")[0, 0] == 2**31 - 2
    Cin = np.array([[5]], dtype=np.int32)
    assert om.matmul(A, B, "i32", Cin=Cin)[0, 0] == -(2**30) + 5


def test_bf16_decode_exact_values():
    # 0x3F80 = 1.0, 0xC000 = -2.0, 0x3F00 = 0.5, 0x4049 = 3.140625
    A = np.array([[0x3F80, 0xC000]], dtype=np.uint16)
    B = np.array([[0x3F00], [0x4049]], dtype=np.uint16)
    assert om.matmul(A, B, "bf16")[0, 0] == 0.5 - 2.0 * 3.140625


def test_bf16_matches_exact_float_values():
    x = inputs.uniform_f32((7, 11), seed=11)
    y = inputs.uniform_f32((11, 3), seed=12)
    xa, ya = inputs.bf16_bits(x), inputs.bf16_bits(y)
    want = inputs.bf16_bits_to_f32(xa).double().numpy() @ inputs.bf16_bits_to_f32(ya).double().numpy()
    assert np.allclose(om.matmul(xa, ya, "bf16"), want, rtol=1e-13, atol=1e-13)


def test_dot_agrees_with_full_product():
    A = inputs.uniform_f32((9, 21), seed=13)
    B = inputs.uniform_f32((21, 8), seed=14)
    C = om.matmul(A, B, "f32")
    for (i, j) in [(0, 0), (8, 7), (3, 5)]:
        assert om.dot(A, B, i, j, "f32") == C[i, j]
    Ai = inputs.full_range_i32((4, 9), seed=15)
    Bi = inputs.full_range_i32((9, 6), seed=16)
    Ci = om.matmul(Ai, Bi, "i32")
    assert om.dot(Ai, Bi, 3, 5, "i32") == Ci[3, 5]


def test_thread_count_does_not_change_result():
    A = inputs.uniform_f32((64, 70), seed=17)
    B = inputs.uniform_f32((70, 33), seed=18)
    assert np.array_equal(om.matmul(A, B, "f32", nthreads=1), om.matmul(A, B, "f32", nthreads=4))


def test_rejects_inconsistent_shapes():
    with pytest.raises(ValueError):
        om.matmul(np.zeros((2, 3), np.float32), np.zeros((4, 2), np.float32), "f32")
