"""Low-precision storage formats of the mixed-precision range finder, in FP64.

Test infrastructure (see the package header): only tests, smoke() and the
bench's cpu_baseline leg may use it.

The paper runs in double precision throughout; the mixed-precision variant
stores A in a narrower format and keeps the orthonormalizations, the small SVD
and the pivoted QR in FP64 (the re-orthonormalization argument of Sec. 3.2 is
what keeps the narrow passes usable).  The formats are fixed here from their
public definitions, and every rounding decision is taken from the FP64 value:

* BF16 (bfloat16): 1 sign bit, 8 exponent bits (bias 127), 7 stored
  significand bits; round to nearest, ties to even, directly from FP64 (no
  intermediate FP32 rounding).
* FP8 E4M3 as defined by the OCP 8-bit floating point specification (the
  "FN" variant: no infinities): 1 sign bit, 4 exponent bits (bias 7), 3
  significand bits.  Exponent field 0 holds the subnormals m/8 * 2^-6
  (m = 1..7); fields 1..15 hold (1 + m/8) * 2^(e-7), except that the code
  with all exponent and significand bits set (S.1111.111) is NaN, so the
  largest finite value is 1.75 * 2^8 = 448.  Values are rounded to nearest,
  ties to even, and saturated to +-448.
* Per-column scales (FP32): s_j = fl32(max_i |A_ij| / 448) (s_j = 1 for a zero
  column), code_ij = e4m3(A_ij / s_j) with the division in FP64 and s_j
  widened exactly; A is represented by dec(code_ij) * s_j.
"""

import numpy as np

E4M3_MAX = 448.0


def bf16_round(x):
    """Nearest BF16 value (ties to even) of each FP64 entry, as FP64.

    A normal BF16 number with exponent e has the spacing 2^(e-7); frexp gives
    x = f 2^E with f in [0.5, 1), so e = E - 1 and the spacing is 2^(E-8).
    The scaling by a power of two is exact, and rint rounds to nearest even.
    Exponents below the smallest normal (2^-126) use its spacing (the
    subnormal grid)."""
    x = np.asarray(x, dtype=np.float64)
    _, E = np.frexp(x)
    E = np.maximum(E, -125)
    q = np.ldexp(1.0, E - 8)
    return np.rint(x / q) * q


def bf16_bits(x):
    """uint16 bit patterns of bf16_round(x) (the upper half of the FP32
    encoding of the same value, which is exact)."""
    v = bf16_round(x).astype(np.float32)
    return (v.view(np.uint32) >> 16).astype(np.uint16)


def e4m3_decode(codes):
    """FP64 value of each E4M3 code (uint8), per the definition above."""
    c = np.asarray(codes, dtype=np.uint8).astype(np.int64)
    s = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 0x7
    sub = m / 8.0 * 2.0 ** -6
    nor = (1.0 + m / 8.0) * np.ldexp(1.0, e - 7)
    v = np.where(e == 0, sub, nor)
    v = np.where((e == 15) & (m == 7), np.nan, v)
    return s * v


def e4m3_encode(y):
    """E4M3 code (uint8) of the nearest value to each FP64 entry of y, ties to
    even, saturated to +-448; NaN gives the NaN code 0x7F.

    For |y| >= 2^-6 (normal range) the spacing is 2^(e-3) with e the binary
    exponent of |y|; below it the spacing is the subnormal 2^-9.  The rounded
    magnitude q * spacing is then re-read as (exponent, significand) fields.
    """
    y = np.asarray(y, dtype=np.float64)
    neg = np.signbit(y)
    a = np.abs(y)
    nan = np.isnan(a)
    a = np.where(nan, 0.0, np.minimum(a, E4M3_MAX))
    _, E = np.frexp(a)                       # a = f 2^E, f in [0.5, 1): exponent e = E - 1
    e = np.maximum(E - 1, -6)
    step = np.ldexp(1.0, e - 3)
    q = np.rint(a / step) * step             # exact scaling, RNE
    q = np.minimum(q, E4M3_MAX)
    # fields of q: normal if q >= 2^-6
    _, E2 = np.frexp(q)
    e2 = E2 - 1
    normal = q >= 2.0 ** -6
    mant_n = np.rint((np.ldexp(q, -np.where(normal, e2, 0)) - 1.0) * 8.0)
    code_n = ((e2 + 7) << 3) + mant_n.astype(np.int64)
    code_s = np.rint(q / 2.0 ** -9).astype(np.int64)
    code = np.where(normal, code_n, code_s).astype(np.int64)
    code = np.where(neg, code | 0x80, code)
    code = np.where(nan, 0x7F, code)
    return code.astype(np.uint8)


def column_scales(A):
    """s_j = fl32(max_i |A_ij| / 448), 1 for an all-zero column (FP32)."""
    A = np.asarray(A, dtype=np.float64)
    mx = np.max(np.abs(A), axis=0)
    s = (mx / E4M3_MAX).astype(np.float32)
    return np.where(mx == 0.0, np.float32(1.0), s).astype(np.float32)


def e4m3_quantize_columns(A):
    """(codes, scales): codes_ij = e4m3(A_ij / s_j) with s = column_scales(A)."""
    A = np.asarray(A, dtype=np.float64)
    s = column_scales(A)
    return e4m3_encode(A / s.astype(np.float64)[None, :]), s


def e4m3_dequantize_columns(codes, scales):
    """A_ij ~ dec(codes_ij) * s_j, in FP64 (the product is exact)."""
    return e4m3_decode(codes) * np.asarray(scales, dtype=np.float64)[None, :]
