"""bfloat16 splitting of float32 values by integer bit operations.

TEST INFRASTRUCTURE ONLY (see the package header).

Not from the paper: the split-precision products are an implementation
choice for MI355X matrix cores.  A float32 value x is written as
    x ~ hi + lo (+ lo2),  hi = bf16(x), lo = bf16(x - hi), lo2 = bf16(x - hi - lo),
with bf16(.) round-to-nearest-even to 8 significant bits.  Each difference is
exact in float32 (it is a multiple of the float32 spacing of x and no larger
than half a bfloat16 spacing), so the three parts carry 24 significant bits.

Products of split values accumulate in float32:
  two-term split   a*b ~ ah*bh + ah*bl + al*bh                    (3 products)
  three-term split a*b ~ ah*bh + ah*bl + al*bh + ah*bl2 + al2*bh + al*bl
                                                                   (6 products)
"""
from __future__ import annotations

import numpy as np


def bf16_bits(x) -> np.ndarray:
    """Upper 16 bits of the round-to-nearest-even bfloat16 of float32 x (no
    NaN inputs): add 0x7FFF plus the lowest kept bit, then truncate."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = (u + 0x7FFF + lsb) >> 16
    return (r & 0xFFFF).astype(np.uint16)


def bf16_value(bits) -> np.ndarray:
    """float32 value of bfloat16 bit patterns."""
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32)


def split(x, parts: int = 2):
    """Split float32 x into ``parts`` bfloat16 bit arrays (hi, lo[, lo2])."""
    x = np.asarray(x, dtype=np.float32)
    out = []
    rem = x.copy()
    for _ in range(parts):
        b = bf16_bits(rem)
        out.append(b)
        rem = (rem - bf16_value(b)).astype(np.float32)
    return out


def split_matmul(A, B, parts: int):
    """float32-accumulated product of split operands (float64 result of the
    float32 sums is returned for comparison).  A: (m, k), B: (k, n)."""
    sa = [bf16_value(p).astype(np.float32) for p in split(A, parts)]
    sb = [bf16_value(p).astype(np.float32) for p in split(B, parts)]
    if parts == 1:
        pairs = [(0, 0)]
    elif parts == 2:
        pairs = [(0, 0), (0, 1), (1, 0)]
    else:
        pairs = [(0, 0), (0, 1), (1, 0), (0, 2), (2, 0), (1, 1)]
    acc = np.zeros((A.shape[0], B.shape[1]), dtype=np.float32)
    for i, j in pairs:
        acc = acc + (sa[i] @ sb[j]).astype(np.float32)
    return acc
