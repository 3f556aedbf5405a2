"""FP8 E4M3 storage (OCP "FN" encoding) for network activations, written from
the format's definition.  Test infrastructure only (see ``oracle/__init__``).

A code is sign | exponent (4 bits, bias 7) | mantissa (3 bits).  Exponent 0
holds the subnormals m * 2^-9; exponents 1..15 hold (1 + m/8) * 2^(e-7),
except that exponent 15 with mantissa 7 is NaN (there is no infinity), so the
largest finite magnitude is 1.75 * 2^8 = 448.

``round_e4m3`` rounds FP64 values to the nearest representable value, ties to
the even code; finite values beyond the range and infinities saturate to
+-448 (reading: activations must stay finite); NaN stays NaN.
"""
from __future__ import annotations

import numpy as np


def e4m3_values() -> np.ndarray:
    """Value of every code 0..255 (NaN for the two NaN codes), FP64."""
    out = np.empty(256)
    for c in range(256):
        s = -1.0 if c & 0x80 else 1.0
        e, m = (c >> 3) & 0xF, c & 7
        if e == 15 and m == 7:
            out[c] = np.nan
        elif e == 0:
            out[c] = s * m * 2.0 ** -9
        else:
            out[c] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return out


def round_e4m3_codes(x) -> np.ndarray:
    """Codes (uint8) of ``x`` rounded to E4M3: nearest magnitude on the
    positive grid, ties to the even code, saturation at 448."""
    x = np.asarray(x, np.float64)
    vals = e4m3_values()[:127]                   # codes 0..126: 0 .. 448, increasing
    a = np.abs(x)
    hi = np.searchsorted(vals, a, side="left")   # first grid value >= a
    hi = np.minimum(hi, 126)
    lo = np.maximum(hi - 1, 0)
    dlo, dhi = a - vals[lo], vals[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(a >= vals[126], 126, np.where(pick_hi, hi, lo))
    code = np.where(a <= 0, 0, code)
    code = code.astype(np.uint8) | np.where(np.signbit(x), 0x80, 0).astype(np.uint8)
    return np.where(np.isnan(x), np.uint8(0x7F), code).astype(np.uint8)


def round_e4m3(x) -> np.ndarray:
    """``x`` rounded to E4M3 and read back as FP64."""
    return e4m3_values()[round_e4m3_codes(x)]


def store_mean_e4m3(sums, counts) -> np.ndarray:
    """Stored E4M3 value of a mean of E4M3 values: the sum of at most eight
    E4M3 values is exact in FP32, the quotient is taken in FP32 (the
    precision of the kernel's arithmetic), then rounded to E4M3."""
    s32 = np.asarray(sums, np.float64).astype(np.float32)
    if not np.array_equal(s32.astype(np.float64), np.asarray(sums, np.float64)):
        raise ValueError("sum of E4M3 children not exact in FP32")
    q = s32 / np.asarray(counts).astype(np.float32)
    return round_e4m3(q.astype(np.float64))
