"""Pins of the oracle's BF16 and FP8-E4M3 encoders by the formats' definitions
(OCP 8-bit floating point, E4M3: bias 7, subnormals, S.1111.111 = NaN, largest
finite 448) and by torch's own BF16 conversion."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth


def test_e4m3_decode_table_from_format():
    t = oracle.e4m3_decode_table()
    assert t[0x00] == 0.0 and t[0x80] == 0.0 and math.copysign(1, t[0x80]) < 0
    assert t[0x01] == 2.0 ** -9            # smallest subnormal
    assert t[0x07] == 7 * 2.0 ** -9        # largest subnormal
    assert t[0x08] == 2.0 ** -6            # smallest normal
    assert t[0x38] == 1.0                  # exponent field 7 = bias
    assert t[0x3C] == 1.5
    assert t[0x7E] == 448.0 and t[0xFE] == -448.0
    assert math.isnan(t[0x7F]) and math.isnan(t[0xFF])
    finite = t[:0x7F]
    assert (np.diff(finite) > 0).all()     # codes 0..126 increase strictly
    for c in range(0x80):
        if c != 0x7F:
            assert t[c | 0x80] == -t[c]
    # 8 values per binade: spacing doubles each binade from 2^-6 on
    for e in range(1, 15):
        vals = t[e * 8:(e + 1) * 8]
        assert np.allclose(np.diff(vals), 2.0 ** (e - 7 - 3))


def test_e4m3_encode_round_to_nearest_even_and_saturate():
    t = oracle.e4m3_decode_table()
    # exact codes round-trip
    for c in list(range(0x7F)) + list(range(0x80, 0xFF)):
        assert oracle.e4m3_encode(np.float32(t[c]))[()] == c or (t[c] == 0.0)
    # midpoints go to the even code
    for c in range(0x00, 0x7E):
        mid = (float(t[c]) + float(t[c + 1])) / 2.0
        got = int(oracle.e4m3_encode(np.float32(mid))[()])
        assert got == (c if c % 2 == 0 else c + 1)
    assert int(oracle.e4m3_encode(np.float32(1000.0))[()]) == 0x7E
    assert int(oracle.e4m3_encode(np.float32(-470.0))[()]) == 0xFE
    assert int(oracle.e4m3_encode(np.float32(2.0 ** -11))[()]) == 0x00  # below half the step
    # random values: the encoding is the nearest code
    x = synth.small_float(21, 1, 3000)[0] * 50
    codes = oracle.e4m3_encode(x)
    for v, c in zip(x, codes):
        d = abs(t[:0x7F] - abs(v))
        assert abs(t[c & 0x7F] - abs(v)) == d.min()


def test_fp8_rows_scale():
    x = synth.small_float(22, 20, 37) * 3
    x[4] = 0.0
    codes, scale = oracle.fp8_encode_rows(x)
    assert scale[4] == 1.0 and (codes[4] & 0x7F == 0).all()
    for i in range(20):
        if i != 4:
            assert scale[i] == np.float32(np.abs(x[i]).max()) / np.float32(448.0)
    dec = oracle.fp8_decode_rows(codes, scale, 37)
    rel = np.abs(dec - x).max(1) / np.abs(x).max(1).clip(1e-30)
    assert (rel[np.arange(20) != 4] <= 2.0 ** -4 + 1e-6).all()  # half a step at 3 mantissa bits


def test_bf16_matches_torch():
    x = synth.small_float(23, 1, 100000)[0] * 1000
    x[:4] = [0.0, -0.0, 1.0, 3.0000002]
    ours = oracle.bf16_encode(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert (ours == ref).all()
    ints = np.arange(256, dtype=np.float32)
    assert (oracle.bf16_decode(oracle.bf16_encode(ints)) == ints).all()  # 0..255 are exact
