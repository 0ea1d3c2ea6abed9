"""Python access to the C oracle of polynomial division modulo a prime (test
infrastructure only).  Definition: Section 5, Fig. 8 -- schoolbook division
of a (N coefficients) by a monic b of degree M given by its M low
coefficients, residues in [0, P)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import build as _build

_fn = None


def _load():
    global _fn
    if _fn is None:
        lib = ctypes.CDLL(_build.build(force=False))
        f = lib.oracle_polydiv_u32
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32]
        _fn = f
    return _fn


def polydiv(a, b, P: int) -> np.ndarray:
    """Returns the dividend array after the division (a copy): its first
    min(N, M) entries are the remainder, the rest zero."""
    try:
        import torch
        if isinstance(a, torch.Tensor):
            a = a.detach().cpu().contiguous().numpy()
        if isinstance(b, torch.Tensor):
            b = b.detach().cpu().contiguous().numpy()
    except ImportError:  # pragma: no cover
        pass
    a = np.array(a, dtype=np.uint32, copy=True).reshape(-1)
    b = np.ascontiguousarray(b, dtype=np.uint32).reshape(-1)
    pa = ctypes.c_void_p(a.ctypes.data if a.size else 0)
    if _load()(pa, a.size, ctypes.c_void_p(b.ctypes.data), b.size, P) != 0:
        raise ValueError("oracle rejected the arguments")
    return a
