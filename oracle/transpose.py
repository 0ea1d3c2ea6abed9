"""Python access to the C oracle of matrix transposition (test infrastructure
only).  Definition: Section 5.2 (Fig. 7, Table 3), C[j][i] = A[i][j]."""
from __future__ import annotations

import ctypes

import numpy as np

from . import build as _build

_fn = None


def _load():
    global _fn
    if _fn is None:
        lib = ctypes.CDLL(_build.build(force=False))
        f = lib.oracle_transpose_u32
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                      ctypes.c_int64]
        _fn = f
    return _fn


def transpose(A) -> np.ndarray:
    """A (M x N) of any 4-byte dtype -> its transpose (N x M), same dtype."""
    try:
        import torch
        if isinstance(A, torch.Tensor):
            A = A.detach().cpu().contiguous().numpy()
    except ImportError:  # pragma: no cover
        pass
    A = np.ascontiguousarray(A)
    if A.dtype.itemsize != 4:
        raise ValueError("4-byte elements only")
    M, N = A.shape
    C = np.empty((N, M), dtype=A.dtype)
    rc = _load()(ctypes.c_void_p(A.ctypes.data if A.size else 0), N,
                 ctypes.c_void_p(C.ctypes.data if C.size else 0), M, M, N)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return C
