"""Rounding to bfloat16, IEEE half precision and FP8 E4M3 (oracle; test infrastructure only).

Used to emulate the reduced-precision MLP paths: values are rounded to the target format with
round-to-nearest-even directly from their float64 value, then all arithmetic continues in float64.

bfloat16: 8 significant bits, 8 exponent bits (float32's range).
half (IEEE binary16, the precision the paper runs its networks in): 11 significant bits, smallest
normal 2^-14, subnormal step 2^-24, largest finite 65504; values that round beyond it become +-inf.
FP8 E4M3 (OCP "E4M3FN"): 4 significant bits, exponent bias 7, smallest normal 2^-6, subnormal step
2^-9, largest finite 448, no infinities; conversion saturates to +-448.
"""
from __future__ import annotations

import numpy as np


def _round_to_quantum(x, quantum):
    return np.rint(x / quantum) * quantum


def round_bf16(x):
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                         # x = m * 2^e, 0.5 <= |m| < 1
    e = np.maximum(e, -125)                    # bf16 subnormals share the 2^-133 step
    q = np.ldexp(1.0, e - 8)
    out = _round_to_quantum(x, q)
    return np.where(x == 0, x, out)


def round_fp16(x):
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                         # |x| in [2^(e-1), 2^e)
    e = np.maximum(e, -13)                     # subnormals share the 2^-24 step
    q = np.ldexp(1.0, e - 11)
    out = _round_to_quantum(x, q)
    out = np.where(np.abs(out) > 65504.0, np.copysign(np.inf, x), out)
    return np.where(x == 0, x, out)


def round_e4m3(x):
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                         # |x| in [2^(e-1), 2^e)
    e = np.maximum(e - 1, -6)                  # unbiased exponent, subnormals share 2^-9 steps
    q = np.ldexp(1.0, e - 3)
    out = _round_to_quantum(x, q)
    out = np.clip(out, -448.0, 448.0)
    return np.where(x == 0, x, out)


def e4m3_values():
    """All 254 finite E4M3 values (positive and negative, +0 and -0 collapse) as float64, sorted."""
    vals = set()
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        ex = (code >> 3) & 0xF
        mant = code & 7
        if ex == 0xF and mant == 7:
            continue                           # NaN
        if ex == 0:
            v = mant / 8.0 * 2.0 ** -6
        else:
            v = (1.0 + mant / 8.0) * 2.0 ** (ex - 7)
        vals.add(s * v)
    return np.array(sorted(vals))
