"""Python access to the C oracle of matrix addition (test infrastructure
only).  Definition: Section 1 (Fig. 1, Fig. 2), C = A + B elementwise."""
from __future__ import annotations

import ctypes

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(_build.build(force=False))
        for name in ("oracle_madd_i32", "oracle_madd_f32"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                          ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        _lib = lib
    return _lib


def madd(A, B, dtype: str) -> np.ndarray:
    try:
        import torch
        if isinstance(A, torch.Tensor):
            A = A.detach().cpu().contiguous().numpy()
        if isinstance(B, torch.Tensor):
            B = B.detach().cpu().contiguous().numpy()
    except ImportError:  # pragma: no cover
        pass
    npt = {"i32": np.int32, "f32": np.float32}[dtype]
    A = np.ascontiguousarray(A, dtype=npt)
    B = np.ascontiguousarray(B, dtype=npt)
    if A.shape != B.shape:
        raise ValueError("shapes differ")
    M, N = A.shape
    C = np.empty((M, N), dtype=npt)
    fn = getattr(_load(), "oracle_madd_" + dtype)
    p = lambda a: ctypes.c_void_p(a.ctypes.data if a.size else 0)
    if fn(p(A), N, p(B), N, p(C), N, M, N) != 0:
        raise ValueError("oracle rejected the arguments")
    return C
