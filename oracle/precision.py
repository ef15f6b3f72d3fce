"""Oracle for the reduced-precision product forms (values stored in FP32 or bfloat16, FP32 x, y
and accumulation).  Test infrastructure only.

The paper never states a value precision; these forms, and their error bounds, follow the usual
floating-point model: every rounding to a format with unit roundoff u satisfies
fl(v) = v (1 + d), |d| <= u.
"""
import math

import numpy as np

U32 = 2.0 ** -24   # FP32 unit roundoff (24-bit significand, round to nearest)
UBF16 = 2.0 ** -8  # bfloat16 unit roundoff (8-bit significand, round to nearest)


def round_f32(v):
    """Round float64 values to FP32 (round to nearest even), returned as float64."""
    return np.asarray(v, np.float64).astype(np.float32).astype(np.float64)


def round_bf16(v):
    """Round float64 values to bfloat16 (8 significant bits, round to nearest, ties to even),
    returned as float64.  Written from the definition: in the binade [2^(e-1), 2^e) representable
    values are multiples of 2^(e-8), and below the smallest normal 2^-126 multiples of the
    subnormal spacing 2^-133; the nearest multiple is taken, ties to the even one.  A result
    beyond the largest finite value, (2 - 2^-7) 2^127, is an infinity of the same sign."""
    v = np.asarray(v, np.float64)
    out = np.zeros_like(v)
    nz = v != 0
    m, e = np.frexp(v[nz])          # v = m 2^e, 0.5 <= |m| < 1
    q = np.ldexp(1.0, np.maximum(e, -125) - 8)  # spacing of representable values there
    r = np.rint(v[nz] / q) * q      # np.rint rounds halves to even
    out[nz] = np.where(np.abs(r) >= 2.0 ** 128, np.copysign(np.inf, r), r)
    out[~nz] = v[~nz]               # +0 and -0 kept
    return out


def bf16_bits(v):
    """16-bit patterns of round_bf16(v) (upper half of the float32 encoding)."""
    f = round_bf16(v).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def gamma(k, u=U32):
    """Higham's gamma_k = k u / (1 - k u): bound of the relative error of k rounded operations."""
    ku = k * u
    return ku / (1.0 - ku) if ku < 1 else math.inf


def dot_error_bound(row_len, u_value):
    """Worst-case |y_i - y_exact_i| / s_i for a row of row_len products in FP32 arithmetic with
    values rounded with unit roundoff u_value and x rounded to FP32 (s_i = sum |a_ik x_k|):
    input roundings (u_value + u32 + u_value u32) plus gamma_k of the k products and k-1 sums,
    each inflated by the input roundings."""
    k = np.asarray(row_len, np.float64)
    g = k * U32 / (1.0 - k * U32)
    return u_value + U32 + u_value * U32 + g * (1 + u_value) * (1 + U32)
