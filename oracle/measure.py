"""Oracle for the small closed-form pieces: block size rule, break-even count, error metric.
Test infrastructure only.
"""
import math

import numpy as np


def ceil_log2_sqrt(n):
    """Smallest t with 2^t >= sqrt(n), i.e. 4^t >= n (integer arithmetic)."""
    t = 0
    while (1 << (2 * t)) < n:
        t += 1
    return t


def csb_log2_beta_range(n):
    """Equation eq:CSB-BlockSize (Section 3.1): ceil(log2 sqrt n) <= log2 beta <= 3 + that."""
    lo = ceil_log2_sqrt(n)
    return lo, lo + 3


def csb_log2_beta(m, n, lds_bytes=64 * 1024, value_bytes=8):
    """Block size choice (Section 3.1): start from the upper bound of the range and lower it while
    beta > 2^16 (16-bit packed local indices) or the beta-entry output slice does not fit the
    on-chip budget (the paper's "fits comfortably in L2", read here as an LDS budget).  The range
    uses max(m, n).  When the budget forces beta below the range, the budget wins."""
    lo, hi = csb_log2_beta_range(max(m, n))
    k = hi
    while k > 0 and ((1 << k) > (1 << 16) or (1 << k) * value_bytes > lds_bytes):
        k -= 1
    return k


def break_even(conv_fmt, conv_crs, spmv_crs, spmv_fmt):
    """Number of products after which a format pays for its extra conversion time
    (Section 7 gives 26, 420, 472 and 1525 without a formula; this is the count N at which
    conv_fmt + N*spmv_fmt = conv_crs + N*spmv_crs).  Inf when the format is not faster; 0 when it
    is faster and converts no slower (it is ahead from the first product)."""
    gain = spmv_crs - spmv_fmt
    if gain <= 0:
        return math.inf
    if conv_fmt <= conv_crs:
        return 0.0
    return (conv_fmt - conv_crs) / gain


def break_even_from_ratios(c_fmt, c_crs, s_crs, s_fmt):
    """Same count in the paper's units: conversion costs C in ParCRS products, speedups S over
    sequential CRS.  With times T_par = T_seq / s_crs and T_fmt = T_seq / s_fmt it reduces to
    (C_fmt - C_crs) / (1 - s_crs / s_fmt)."""
    t_seq = 1.0
    t_par = t_seq / s_crs
    return break_even(c_fmt * t_par, c_crs * t_par, t_par, t_seq / s_fmt)


def scaled_error(y, y_ref, scale):
    """Row-scaled error |y - y_ref| / scale per row; rows with scale 0 give 0 when y is +-0 and
    inf otherwise."""
    y = np.asarray(y, np.float64)
    d = np.abs(y - np.asarray(y_ref, np.float64))
    s = np.asarray(scale, np.float64)
    out = np.zeros_like(d)
    pos = s > 0
    out[pos] = d[pos] / s[pos]
    out[~pos] = np.where(y[~pos] == 0.0, 0.0, np.inf)
    return out


def equal_ignoring_zero_sign(a, b):
    """Bitwise equality of float64 arrays where -0.0 and +0.0 count as equal."""
    a = np.asarray(a, np.float64) + 0.0
    b = np.asarray(b, np.float64) + 0.0
    return np.array_equal(a.view(np.int64), b.view(np.int64))
