"""Reduced-precision Gram blocks (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The method itself is stated in exact arithmetic; the tall-skinny products of Section 3
(X^T X, X^T G, G^T G and their B-metric forms) are where a bfloat16 mode rounds its
operands.  This module states what such a product is, from the definitions:

* bfloat16 keeps 8 significant bits of a binary32 value and its exponent range; rounding is
  to nearest with ties to even;
* the product of two bfloat16 values has at most 16 significant bits, so the Gram blocks of
  the rounded operands are exact in FP64 up to the order of the sum.
"""
from __future__ import annotations

import numpy as np


def round_bf16(x):
    """Nearest bfloat16 value of each entry (ties to even), as float64.

    x = m 2^e with m in [0.5, 1): the significand m 2^8 is rounded to an integer (ties to
    even) and scaled back.  Finite inputs in the normal binary32 range only."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.rint(m * 256.0), e - 8)


def gram_blocks_bf16(A, B):
    """[A^T A, A^T B, B^T B] of the bfloat16-rounded blocks, in FP64."""
    Ar, Br = round_bf16(A), round_bf16(B)
    return Ar.T @ Ar, Ar.T @ Br, Br.T @ Br
