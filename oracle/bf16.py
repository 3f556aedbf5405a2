"""BF16 storage of particle and tree values, written from the format's
definition.  Test infrastructure only (see ``oracle/__init__``).

BF16 keeps the sign and the 8-bit exponent of IEEE binary32 and 7 stored
fraction bits: a normal value is (1 + m/128) * 2^e with the exponent range of
binary32, subnormals are multiples of 2^-133.  ``round_bf16`` rounds to the
nearest representable value with ties to the even fraction (the rounding of
the library's stores); magnitudes past the largest finite value round to
infinity as in binary32.

The library computes every tree mean in FP32 and stores each level's means
in the storage type, and the next coarser level averages the stored values.
``store_mean_bf16`` is that storage rule, for ``oracle.tree.fill_tree``'s
``store`` hook.
"""
from __future__ import annotations

import numpy as np

BF16_MAX = (2.0 - 2.0 ** -7) * 2.0 ** 127


def round_bf16(x) -> np.ndarray:
    """``x`` (FP64 holding FP32 values, or FP32) rounded to BF16, as FP64."""
    x = np.asarray(x, np.float64)
    out = np.array(x, np.float64, copy=True)
    fin = np.isfinite(x) & (x != 0)
    a = np.abs(x[fin])
    _, e = np.frexp(a)                       # a = f * 2^e, f in [0.5, 1)
    # spacing of the BF16 grid around a: 8 significant bits for normal
    # values (2^(e-8)), the subnormal spacing 2^-133 below 2^-126
    step = np.ldexp(1.0, np.maximum(e - 8, -133))
    q = np.rint(a / step)                    # round half to even on the grid index
    r = q * step
    r = np.where(r > BF16_MAX, np.inf, r)
    out[fin] = np.copysign(r, x[fin])
    return out


def store_mean_bf16(sums, counts) -> np.ndarray:
    """Stored BF16 value of a mean of BF16 values: the children's sum must
    be exact in FP32 (then the order of the sum does not matter), the
    quotient is taken in FP32 (the arithmetic of the fill), then rounded to
    BF16."""
    s = np.asarray(sums, np.float64)
    s32 = s.astype(np.float32)
    if not np.array_equal(s32.astype(np.float64), s):
        raise ValueError("sum of BF16 children not exact in FP32")
    q = s32 / np.asarray(counts).astype(np.float32)
    return round_bf16(q.astype(np.float64))
