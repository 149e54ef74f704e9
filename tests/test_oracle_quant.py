"""Pins of the oracle's low-precision formats (oracle/quant.py), against
torch's independent implementations of the same public formats and against
properties fixed by the definitions (no GPU needed).

* The 256-code E4M3 table equals torch.float8_e4m3fn's decoding of the same
  bytes (NaN at 0x7F and 0xFF, largest finite 448).
* Encoding: every finite code round-trips; random FP32 values in range and the
  exact midpoints between neighbouring codes encode as torch's conversion does
  (round to nearest, ties to even); out-of-range values saturate to +-448.
* BF16: equal to torch's FP32 -> bfloat16 rounding on FP32 inputs (ties
  included), and rounded directly from FP64 where rounding through FP32
  first would differ (no double rounding).
* Per-column scaling: each nonzero column's largest entry maps to code
  magnitude 448, and dequantization is within half a code step of A.
"""

import numpy as np
import torch

from oracle import quant as QZ


def torch_e4m3_table():
    b = torch.arange(256, dtype=torch.int64).to(torch.uint8)
    return b.view(torch.float8_e4m3fn).to(torch.float64).numpy()


def test_e4m3_decode_table_matches_torch():
    ref = torch_e4m3_table()
    got = QZ.e4m3_decode(np.arange(256, dtype=np.uint8))
    nan_r, nan_g = np.isnan(ref), np.isnan(got)
    assert np.array_equal(nan_r, nan_g)
    assert np.array_equal(np.flatnonzero(nan_g), [0x7F, 0xFF])
    assert np.array_equal(got[~nan_g], ref[~nan_r])
    assert np.nanmax(got) == 448.0 and np.nanmin(got) == -448.0
    assert got[1] == 2.0 ** -9 and got[8] == 2.0 ** -6     # smallest subnormal, normal


def test_e4m3_roundtrip_every_finite_code():
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], dtype=np.uint8)
    assert np.array_equal(QZ.e4m3_encode(QZ.e4m3_decode(codes)), codes)


def _torch_encode(x32):
    t = torch.from_numpy(x32.astype(np.float32)).to(torch.float8_e4m3fn)
    return t.view(torch.uint8).numpy()


def test_e4m3_encode_matches_torch_random():
    g = np.random.default_rng(3)
    x = np.concatenate([g.uniform(-448, 448, 20000),
                        g.standard_normal(20000) * 2.0 ** g.integers(-12, 8, 20000),
                        g.uniform(-2.0 ** -6, 2.0 ** -6, 5000)]).astype(np.float32)
    got = QZ.e4m3_encode(x.astype(np.float64))
    ref = _torch_encode(x)
    # -0.0 and +0.0: torch keeps the sign of zero too
    assert np.array_equal(got, ref)


def test_e4m3_encode_ties_to_even():
    vals = QZ.e4m3_decode(np.arange(0x7E + 1, dtype=np.uint8))   # 0 .. 448, increasing
    mid = (vals[:-1] + vals[1:]) / 2.0                           # exact in FP64 and FP32
    got = QZ.e4m3_encode(mid)
    ref = _torch_encode(mid.astype(np.float32))
    assert np.array_equal(got, ref)
    lo = np.arange(0x7E, dtype=np.uint8)
    # ties go to the code with an even significand field
    assert np.all(got % 2 == 0)
    assert np.all((got == lo) | (got == lo + 1))


def test_e4m3_saturates_and_nan():
    assert QZ.e4m3_encode(np.array([448.0, 464.0, 1e9]))[0] == 0x7E
    assert np.all(QZ.e4m3_encode(np.array([448.0, 464.0, 1e9])) == 0x7E)
    assert np.all(QZ.e4m3_encode(np.array([-500.0, -1e300])) == 0xFE)
    assert QZ.e4m3_encode(np.array([np.nan]))[0] == 0x7F


def test_bf16_matches_torch_on_fp32_inputs():
    g = np.random.default_rng(5)
    x = (g.standard_normal(50000) * 10.0 ** g.integers(-8, 8, 50000)).astype(np.float32)
    # exact BF16 midpoints: low 16 bits = 0x8000
    bits = (g.integers(0, 2 ** 31, 5000, dtype=np.uint64).astype(np.uint32) & 0x7FFF0000) | 0x8000
    x = np.concatenate([x, bits.view(np.float32)])
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = QZ.bf16_round(x.astype(np.float64))
    assert np.array_equal(got, ref)
    assert np.array_equal(QZ.bf16_bits(x.astype(np.float64)),
                          torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy()
                          .astype(np.uint16))


def test_bf16_rounds_directly_from_fp64():
    # 1 + 2^-8 is the midpoint between the BF16 neighbours 1 and 1 + 2^-7; a
    # value just above it rounds up, but rounding to FP32 first lands exactly on
    # the midpoint and then ties to even (down to 1)
    x = 1.0 + 2.0 ** -8 + 2.0 ** -40
    assert float(np.float32(x)) == 1.0 + 2.0 ** -8
    assert QZ.bf16_round(np.array([x]))[0] == 1.0 + 2.0 ** -7
    assert QZ.bf16_round(np.array([1.0 + 2.0 ** -8]))[0] == 1.0


def test_column_scales_and_dequantization():
    g = np.random.default_rng(9)
    A = g.standard_normal((300, 40)) * np.logspace(-3, 2, 40)[None, :]
    A[:, 7] = 0.0
    codes, s = QZ.e4m3_quantize_columns(A)
    assert s.dtype == np.float32 and s[7] == 1.0
    mag = codes & 0x7F
    for j in range(40):
        if j == 7:
            assert np.all(mag[:, j] == 0)
        else:
            assert mag[:, j].max() == 0x7E
    D = QZ.e4m3_dequantize_columns(codes, s)
    # relative half-step of a 3-bit significand (subnormals: absolute 2^-10 s)
    err = np.abs(D - A)
    bound = np.maximum(np.abs(A) * 2.0 ** -4, 2.0 ** -10 * s.astype(np.float64)[None, :])
    assert np.all(err <= bound * (1 + 1e-12))
