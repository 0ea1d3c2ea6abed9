"""Python access to the C oracle of the matrix product (test infrastructure only).

Definition followed: Section 2, Fig. 3 (blocked product whose innermost
statement accumulates a[p][k]*b[k][q] into c[p][q]), written out for
rectangular row-major operands; see ``oracle/matmul.c`` for the arithmetic.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        for name in ("oracle_matmul_f32", "oracle_matmul_bf16", "oracle_matmul_i32"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [vp, i64, vp, i64, vp, vp, i64, i64, i64, i64, i32, i32]
        for name, rt in (("oracle_dot_f32", ctypes.c_double), ("oracle_dot_bf16", ctypes.c_double),
                         ("oracle_dot_i32", ctypes.c_int32)):
            fn = getattr(lib, name)
            fn.restype = rt
            fn.argtypes = [vp, i64, vp, i64, i64, i64, i64]
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else ctypes.c_void_p(0)


def threads() -> int:
    """Number of OpenMP threads the oracle uses by default."""
    return _load().oracle_threads()


def _as_np(x):
    try:
        import torch
        if isinstance(x, torch.Tensor):
            return x.detach().cpu().contiguous().numpy()
    except ImportError:  # pragma: no cover
        pass
    return np.ascontiguousarray(x)


def matmul(A, B, dtype: str, Cin=None, nthreads: int = 0) -> np.ndarray:
    """C = (Cin if given) + A @ B by the oracle.

    ``dtype`` names how the input bytes are read: ``"f32"`` (float32),
    ``"bf16"`` (uint16/int16 bfloat16 bit patterns) or ``"i32"`` (int32,
    wrapping).  Returns float64 for f32/bf16 and int32 for i32.
    """
    A = _as_np(A)
    B = _as_np(B)
    M, K = A.shape
    K2, N = B.shape
    if K2 != K:
        raise ValueError("inner dimensions differ: %d vs %d" % (K, K2))
    lib = _load()
    acc = 1 if Cin is not None else 0
    if dtype == "f32":
        A = np.ascontiguousarray(A, dtype=np.float32)
        B = np.ascontiguousarray(B, dtype=np.float32)
        C = np.zeros((M, N), dtype=np.float64)
        cin = np.ascontiguousarray(_as_np(Cin), dtype=np.float64) if acc else None
        rc = lib.oracle_matmul_f32(_ptr(A), K, _ptr(B), N, _ptr(cin), _ptr(C), N, M, N, K, acc, nthreads)
    elif dtype == "bf16":
        A = np.ascontiguousarray(A).view(np.uint16)
        B = np.ascontiguousarray(B).view(np.uint16)
        C = np.zeros((M, N), dtype=np.float64)
        cin = np.ascontiguousarray(_as_np(Cin), dtype=np.float64) if acc else None
        rc = lib.oracle_matmul_bf16(_ptr(A), K, _ptr(B), N, _ptr(cin), _ptr(C), N, M, N, K, acc, nthreads)
    elif dtype == "i32":
        A = np.ascontiguousarray(A, dtype=np.int32)
        B = np.ascontiguousarray(B, dtype=np.int32)
        C = np.zeros((M, N), dtype=np.int32)
        cin = np.ascontiguousarray(_as_np(Cin), dtype=np.int32) if acc else None
        rc = lib.oracle_matmul_i32(_ptr(A), K, _ptr(B), N, _ptr(cin), _ptr(C), N, M, N, K, acc, nthreads)
    else:
        raise ValueError("unknown dtype %r" % dtype)
    if rc != 0:
        raise ValueError("oracle rejected the arguments (rc=%d)" % rc)
    return C


def dot(A, B, i: int, j: int, dtype: str):
    """One output element C[i][j] = sum_k A[i][k] * B[k][j] (no Cin)."""
    A = _as_np(A)
    B = _as_np(B)
    M, K = A.shape
    N = B.shape[1]
    lib = _load()
    if dtype == "f32":
        A = np.ascontiguousarray(A, dtype=np.float32)
        B = np.ascontiguousarray(B, dtype=np.float32)
        return lib.oracle_dot_f32(_ptr(A), K, _ptr(B), N, i, j, K)
    if dtype == "bf16":
        A = np.ascontiguousarray(A).view(np.uint16)
        B = np.ascontiguousarray(B).view(np.uint16)
        return lib.oracle_dot_bf16(_ptr(A), K, _ptr(B), N, i, j, K)
    if dtype == "i32":
        A = np.ascontiguousarray(A, dtype=np.int32)
        B = np.ascontiguousarray(B, dtype=np.int32)
        return lib.oracle_dot_i32(_ptr(A), K, _ptr(B), N, i, j, K)
    raise ValueError("unknown dtype %r" % dtype)
