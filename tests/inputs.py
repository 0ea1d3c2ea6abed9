"""Seeded synthetic inputs for the tests, the smoke check and the benchmark.

This module holds random draws and dtype packing only: none of the matrix
product, the case table or the cost model is computed here.  Both the HIP
path and the CPU oracle receive the very same host bytes produced by these
functions, so the random generator never influences parity.

Recipes (all draws use ``torch.Generator`` on the CPU):

* ``uniform_f32``: i.i.d. uniform on [-1, 1): ``rand * 2 - 1`` in float32.
* ``small_int_i32``: i.i.d. integers uniform on [lo, hi] inclusive
  (default [-8, 8]).
* ``full_range_i32``: i.i.d. integers over the whole int32 range, so that
  products and sums wrap modulo 2**32.
* ``bf16_bits``: float32 rounded to bfloat16 with round-to-nearest-even
  (torch's own conversion), returned as the raw uint16 bit patterns.
* ``group_dims``: sizes ``round(exp(U(ln lo, ln hi)))`` for batched problems.
* ``sweep_shapes``: the 216 (M, N, K) triples over {512, 1000, 2048, 3000,
  4096, 8192}^3, with a per-shape seed derived as
  ``seed + 1_000_003 * index`` so every shape has its own stream.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import torch

SWEEP_SIZES = (512, 1000, 2048, 3000, 4096, 8192)


def _gen(seed: int) -> torch.Generator:
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    return g


def uniform_f32(shape, seed: int) -> torch.Tensor:
    """float32 tensor, entries i.i.d. uniform on [-1, 1)."""
    return torch.rand(tuple(shape), generator=_gen(seed), dtype=torch.float32) * 2.0 - 1.0


def small_int_i32(shape, seed: int, lo: int = -8, hi: int = 8) -> torch.Tensor:
    """int32 tensor, entries i.i.d. uniform integers on [lo, hi]."""
    return torch.randint(lo, hi + 1, tuple(shape), generator=_gen(seed), dtype=torch.int32)


def small_int_f32(shape, seed: int, lo: int = -8, hi: int = 8) -> torch.Tensor:
    """float32 tensor holding small integers (exactly representable)."""
    return small_int_i32(shape, seed, lo, hi).to(torch.float32)


def full_range_i32(shape, seed: int) -> torch.Tensor:
    """int32 tensor over the full signed range (wrapping arithmetic case)."""
    x = torch.randint(-(2**31), 2**31, tuple(shape), generator=_gen(seed), dtype=torch.int64)
    return x.to(torch.int32)


def bf16_bits(x_f32: torch.Tensor) -> torch.Tensor:
    """Round float32 to bfloat16 (nearest-even); return the uint16 bit patterns
    stored in an int16 tensor (same bytes)."""
    return x_f32.to(torch.bfloat16).view(torch.int16)


def bf16_bits_to_f32(bits: torch.Tensor) -> torch.Tensor:
    """The exact float32 value of bfloat16 bit patterns."""
    return bits.view(torch.bfloat16).to(torch.float32)


def group_dims(count: int, seed: int, lo: int = 16, hi: int = 512) -> np.ndarray:
    """(count, 3) int64 array of (M, N, K), each round(exp(U(ln lo, ln hi)))."""
    u = torch.rand((count, 3), generator=_gen(seed), dtype=torch.float64).numpy()
    v = np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))
    return np.clip(np.rint(v), lo, hi).astype(np.int64)


def log_uniform_shapes(count: int, seed: int, lo: int = 64, hi: int = 8192) -> np.ndarray:
    """(count, 3) random shapes, log-uniform on [lo, hi]."""
    return group_dims(count, seed, lo, hi)


def sweep_shapes():
    """The 216 (M, N, K) shapes of the FP32 sweep, in a fixed order."""
    return list(itertools.product(SWEEP_SIZES, repeat=3))


def sweep_seed(index: int, seed: int = 0) -> int:
    return seed + 1_000_003 * index
