"""Pins of the oracle's BF16 and e4m3fn storage formats (no GPU)."""
import numpy as np
import pytest
import torch

import oracle


def test_e4m3fn_known_codes():
    t = oracle.e4m3fn_table()
    assert t[0x00] == 0.0 and np.signbit(t[0x80])
    assert t[0x38] == 1.0 and t[0xB8] == -1.0
    assert t[0x7E] == 448.0 and t[0xFE] == -448.0
    assert t[0x01] == 2.0 ** -9                    # smallest subnormal
    assert t[0x07] == 7 / 8 * 2.0 ** -6            # largest subnormal
    assert t[0x08] == 2.0 ** -6                    # smallest normal
    assert np.isnan(t[0x7F]) and np.isnan(t[0xFF])
    assert np.isfinite(np.delete(t, [0x7F, 0xFF])).all()


def test_e4m3fn_table_matches_torch():
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    tv = codes.view(torch.float8_e4m3fn).float().double().numpy()
    t = oracle.e4m3fn_table()
    np.testing.assert_array_equal(np.isnan(t), np.isnan(tv))
    np.testing.assert_array_equal(t[~np.isnan(t)], tv[~np.isnan(tv)])


def test_e4m3fn_encode_matches_torch_in_range():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-440, 440, 20000), rng.standard_normal(20000) * 1e-2,
                        rng.standard_normal(5000) * 1e-3]).astype(np.float32)
    # exact halfway points between neighbouring codes exercise ties-to-even
    mags = oracle.e4m3fn_table()[:127]
    mid = ((mags[:-1] + mags[1:]) / 2).astype(np.float32)
    x = np.concatenate([x, mid, -mid])
    ours = oracle.e4m3fn_encode(x)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(ours, ref)


def test_e4m3fn_saturates_and_round_trips():
    assert oracle.e4m3fn_encode(np.float32(1e6)) == 0x7E
    assert oracle.e4m3fn_encode(np.float32(-1e6)) == 0xFE
    assert oracle.e4m3fn_encode(np.float32(470.0)) == 0x7E
    assert oracle.e4m3fn_encode(np.float32(np.nan)) & 0x7F == 0x7F
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], dtype=np.uint8)
    np.testing.assert_array_equal(oracle.e4m3fn_encode(oracle.e4m3fn_decode(codes)), codes)


def test_bf16_encode_matches_torch():
    rng = np.random.default_rng(2)
    x = (rng.standard_normal(50000) * np.exp(rng.uniform(-20, 20, 50000))).astype(np.float32)
    ties = ((rng.integers(0, 2 ** 15, 2000).astype(np.uint32) << 16) | 0x8000).view(np.float32)
    ties = ties[np.isfinite(ties)]
    x = np.concatenate([x, ties, np.array([0.0, -0.0, 3.0e38, -3.0e38], np.float32)])
    ours = oracle.bf16_encode(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(ours, ref)
    assert oracle.bf16_decode(np.uint16(0x3F80)) == 1.0
    assert np.isnan(oracle.bf16_decode(oracle.bf16_encode(np.array([np.nan], np.float32))))[0]


def test_fp8_rows_quantize_definition():
    rng = np.random.default_rng(3)
    A = (rng.standard_normal((40, 77)) * np.exp(rng.uniform(-5, 5, (40, 1)))).astype(np.float32)
    A[5] = 0.0
    q, s = oracle.fp8_rows_quantize(A)
    assert q.dtype == np.uint8 and s.dtype == np.float32
    assert s[5] == 1.0 and (q[5] == 0).all()
    amax = np.abs(A).max(axis=1)
    # scales are powers of two, the smallest with amax / s <= 448 (so amax / s > 224)
    mant, _ = np.frexp(s.astype(np.float64))
    assert (mant == 0.5).all()
    r = amax[amax > 0] / s[amax > 0].astype(np.float64)
    assert (r <= 448.0).all() and (r > 224.0).all()
    Ad = oracle.fp8_rows_dequantize(q, s)
    # three significand bits: relative error at most 2^-4 above the subnormal range
    big = np.abs(A) >= 2.0 ** -6 * s[:, None]
    rel = np.abs(Ad[big] - A[big]) / np.abs(A[big])
    assert rel.max() <= 2.0 ** -4 * (1 + 1e-6)
    # dequantisation is an exact product by a power of two
    np.testing.assert_array_equal(Ad.astype(np.float64),
                                  oracle.e4m3fn_decode(q).astype(np.float64) * s[:, None].astype(np.float64))
    # the row maximum lands in the top binade of the format
    assert (np.abs(oracle.e4m3fn_decode(q)).max(axis=1)[amax > 0] >= 224).all()


def test_fp8_row_scale_edges():
    # exact boundaries of the rule 448 * 2^k >= amax
    a = np.array([448.0, 448.00003, 224.0, 1.0, 3.0e38, 1e-45, 0.0], dtype=np.float32)
    s = oracle.fp8_row_scale(a)
    assert s[0] == 1.0 and s[1] == 2.0 and s[2] == 0.5
    assert s[3] == 2.0 ** -8               # 448 / 512 = 0.875 < 1 <= 448 / 256
    assert s[4] == 2.0 ** 120              # 3e38 / 2^120 = 225.6
    assert s[5] == np.float32(2.0 ** -126) and s[6] == 1.0
