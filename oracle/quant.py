"""Storage formats for the precision modes: BF16 and OCP FP8 E4M3 (e4m3fn) with row scales.

Test infrastructure only (see the package docstring).  The paper itself stores
everything in full precision; these are the definitions the reduced-storage
modes are checked against: the oracle runs on the dequantised matrix.

Formats, written from their definitions:
  * bfloat16: the upper 16 bits of an IEEE binary32; encoding picks the nearest
    bfloat16 value, ties to the even significand.
  * e4m3fn (OCP 8-bit floating point, E4M3): 1 sign, 4 exponent (bias 7) and
    3 significand bits; exponent field 0 is subnormal; S.1111.111 is NaN; there
    is no infinity; the largest finite magnitude is 448.  Encoding picks the
    nearest finite value, ties to the even code, and saturates to +-448.
  * Per-row scaling by a power of two: s_i = 2^k_i with k_i the smallest integer
    >= -126 such that 448 * 2^k_i >= amax_i (s_i = 1 for an all-zero row), so
    q_ij = e4m3fn(fl32(A_ij / s_i)) never saturates and the dequantised value
    a'_ij = fl32(s_i * q_ij) is the exact product (the hardware's scaled e4m3
    conversion applies exactly such a scale).

Pins (tests/test_oracle_quant.py): known code points of both formats; decode and
encode against torch's CPU float8_e4m3fn / bfloat16 conversions on in-range
values; round trips of every representable value.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


# ------------------------------- bfloat16 -----------------------------------
def bf16_decode(u):
    """bfloat16 bit patterns (uint16) -> float32 values."""
    u = np.asarray(u, dtype=np.uint16)
    return (u.astype(np.uint32) << np.uint32(16)).view(np.float32)


def bf16_encode(x):
    """float32 -> bfloat16 bit patterns, nearest value, ties to even."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    bits = x.view(np.uint32)
    lo = bits & np.uint32(0xFFFF0000)                 # truncated toward zero
    hi = lo + np.uint32(0x10000)                      # next magnitude up
    with np.errstate(over="ignore", invalid="ignore"):
        v = x.astype(np.float64)
        d_lo = np.abs(v - lo.view(np.float32).astype(np.float64))
        d_hi = np.abs(hi.view(np.float32).astype(np.float64) - v)
    lo_even = ((lo >> np.uint32(16)) & np.uint32(1)) == 0
    pick_hi = (d_hi < d_lo) | ((d_hi == d_lo) & ~lo_even)
    out = np.where(pick_hi, hi, lo) >> np.uint32(16)
    out = out.astype(np.uint16)
    nan = np.isnan(x)
    out[nan] = ((bits[nan] >> np.uint32(16)) | np.uint32(0x0040)).astype(np.uint16)
    inf = np.isinf(x)
    out[inf] = (bits[inf] >> np.uint32(16)).astype(np.uint16)
    return out


def bf16_quantize(A):
    return bf16_encode(A)


def bf16_dequantize(u):
    return bf16_decode(u)


# ------------------------------- e4m3fn --------------------------------------
def e4m3fn_table():
    """float64 value of every e4m3fn code 0..255 (NaN for the two NaN codes)."""
    t = np.empty(256, dtype=np.float64)
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        m = code & 0x7
        if e == 0xF and m == 0x7:
            t[code] = np.nan
        elif e == 0:
            t[code] = s * (m / 8.0) * 2.0 ** (1 - 7)
        else:
            t[code] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return t


_TABLE = e4m3fn_table()
_MAGS = _TABLE[:127]          # codes 0x00..0x7E: 0 .. 448, strictly increasing


def e4m3fn_decode(q):
    """e4m3fn codes (uint8) -> float32 values (every finite code is exact in float32)."""
    return _TABLE[np.asarray(q, dtype=np.uint8)].astype(np.float32)


def e4m3fn_encode(x):
    """float32 -> e4m3fn codes: nearest finite value, ties to the even code, saturating."""
    x = np.asarray(x, dtype=np.float32)
    mag = np.abs(x.astype(np.float64))
    neg = np.signbit(x)
    code = np.empty(x.shape, dtype=np.int64)
    big = mag >= E4M3_MAX
    code[big] = 126
    small = ~big & ~np.isnan(x)
    m = mag[small]
    hi = np.searchsorted(_MAGS, m, side="left")       # _MAGS[hi] >= m
    hi = np.clip(hi, 0, 126)
    lo = np.clip(hi - 1, 0, 126)
    d_hi = _MAGS[hi] - m
    d_lo = m - _MAGS[lo]
    exact = d_hi == 0
    pick_hi = exact | (d_hi < d_lo) | ((d_hi == d_lo) & (hi % 2 == 0))
    code[small] = np.where(pick_hi, hi, lo)
    code[np.isnan(x)] = 127
    code = code | np.where(neg, 0x80, 0)
    return code.astype(np.uint8)


def fp8_row_scale(amax):
    """Smallest power of two s = 2^k, k >= -126, with 448 s >= amax (1 when amax is 0).

    With amax = m 2^e, m in [0.5, 1): 448 = 0.875 * 2^9, so k = e - 9 when m <= 0.875
    and k = e - 8 otherwise -- integer logic on the exact binary exponent.
    """
    amax = np.asarray(amax, dtype=np.float32)
    m, e = np.frexp(amax.astype(np.float64))
    k = e.astype(np.int64) - 9 + (m > 0.875).astype(np.int64)
    k = np.maximum(k, -126)
    s = np.ldexp(np.ones_like(m), k).astype(np.float32)
    return np.where(amax == 0, np.float32(1.0), s).astype(np.float32)


def fp8_rows_quantize(A):
    """Row-scaled e4m3fn storage of a float32 matrix -> (codes uint8, scales float32)."""
    A = np.asarray(A, dtype=np.float32)
    amax = np.max(np.abs(A), axis=1).astype(np.float32)
    s = fp8_row_scale(amax)
    t = (A / s[:, None]).astype(np.float32)
    return e4m3fn_encode(t), s


def fp8_rows_dequantize(q, s):
    """a'_ij = fl32(s_i * decode(q_ij))."""
    return (np.asarray(s, dtype=np.float32)[:, None] * e4m3fn_decode(q)).astype(np.float32)
