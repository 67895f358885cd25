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
    np.testing.assert_array_equal(s[amax > 0], (amax / np.float32(448.0)).astype(np.float32)[amax > 0])
    Ad = oracle.fp8_rows_dequantize(q, s)
    # three significand bits: relative error at most 2^-4 above the subnormal range
    big = np.abs(A) >= 2.0 ** -6 * s[:, None]
    rel = np.abs(Ad[big] - A[big]) / np.abs(A[big])
    assert rel.max() <= 2.0 ** -4 * (1 + 1e-6)
    # the row maximum lands on the top code (or its neighbour after the scale's rounding)
    assert (np.abs(oracle.e4m3fn_decode(q)).max(axis=1)[amax > 0] >= 416).all()
