"""Python access to the C oracle of the 1D Jacobi example (test
infrastructure only).  Definition: Section 5, Fig. 6 (source program): T
time steps over an array of 2N elements holding two copies of the vector,
each step averaging three neighbours of one copy into the other."""
from __future__ import annotations

import ctypes

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(_build.build(force=False))
        for name in ("oracle_jacobi1d_i32", "oracle_jacobi1d_f32"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64]
        _lib = lib
    return _lib


def jacobi1d(a, steps: int, dtype: str) -> np.ndarray:
    """a: the 2N-element array (both copies); returns the array after
    `steps` time steps (a copy; the input is not modified)."""
    try:
        import torch
        if isinstance(a, torch.Tensor):
            a = a.detach().cpu().contiguous().numpy()
    except ImportError:  # pragma: no cover
        pass
    npt = {"i32": np.int32, "f32": np.float32}[dtype]
    a = np.array(a, dtype=npt, copy=True).reshape(-1)
    if a.size % 2:
        raise ValueError("the array holds two copies: even length")
    N = a.size // 2
    fn = getattr(_load(), "oracle_jacobi1d_" + dtype)
    if fn(ctypes.c_void_p(a.ctypes.data if a.size else 0), N, steps) != 0:
        raise ValueError("oracle rejected the arguments")
    return a


def result_half(a: np.ndarray, steps: int) -> np.ndarray:
    """The copy the last step wrote: the second after an odd number of steps,
    the first after an even number."""
    N = a.size // 2
    return a[N:] if steps % 2 else a[:N]
