"""Pins of the oracle's BF16 / FP8-E4M3FN encoders, decoders and power-of-two
scales: exhaustive round trips over every code, agreement with torch's own
casts (a library routine), hand-picked ties and boundaries (CPU only)."""
import math

import numpy as np
import pytest
import torch


def test_bf16_roundtrip_all_codes(orc):
    for h in range(0, 1 << 16, 1):
        f = orc.bf16_decode(h)
        if math.isnan(f):
            assert math.isnan(orc.bf16_decode(orc.bf16_encode(f)))
            continue
        assert orc.bf16_encode(f) == h, hex(h)


def test_bf16_matches_torch_cast(orc):
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.uniform(-1, 1, 4000), rng.normal(0, 1e3, 2000), rng.normal(0, 1e-30, 1000),
        np.float32(rng.uniform(-1, 1, 2000)) * np.float32(2.0 ** -130),
        [0.0, -0.0, 3.4e38, -3.4e38, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8],
    ]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    got = np.array([orc.bf16_encode(v) for v in x], dtype=np.uint16)
    np.testing.assert_array_equal(got, ref)


def test_bf16_ties_to_even(orc):
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: even mantissa (1.0) wins
    assert orc.bf16_encode(1.0 + 2 ** -8) == 0x3F80
    # 1 + 3*2^-8 halfway between 1+2^-7 (odd) and 1+2^-6 (even)
    assert orc.bf16_encode(1.0 + 3 * 2 ** -8) == 0x3F82
    assert orc.bf16_encode(float("inf")) == 0x7F80
    assert orc.bf16_encode(-0.0) == 0x8000


def test_e4m3_decode_definition(orc):
    assert orc.e4m3_decode(0x7E) == 448.0
    assert orc.e4m3_decode(0xFE) == -448.0
    assert orc.e4m3_decode(0x08) == 2.0 ** -6
    assert orc.e4m3_decode(0x01) == 2.0 ** -9
    assert orc.e4m3_decode(0x07) == 7 * 2.0 ** -9
    assert orc.e4m3_decode(0x38) == 1.0
    assert orc.e4m3_decode(0x39) == 1.125
    assert math.isnan(orc.e4m3_decode(0x7F)) and math.isnan(orc.e4m3_decode(0xFF))
    vals = [orc.e4m3_decode(c) for c in range(0x7F)]
    assert all(b > a for a, b in zip(vals, vals[1:]))     # codes are monotone


def test_e4m3_roundtrip_all_codes(orc):
    for c in range(256):
        v = orc.e4m3_decode(c)
        if math.isnan(v):
            assert orc.e4m3_encode(v) & 0x7F == 0x7F
            continue
        assert orc.e4m3_encode(v) == c, hex(c)


def test_e4m3_matches_torch_cast_in_range(orc):
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-448, 448, 3000), rng.normal(0, 1, 3000),
                        rng.normal(0, 2 ** -7, 2000)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = np.array([orc.e4m3_encode(float(v)) for v in x], dtype=np.uint8)
    np.testing.assert_array_equal(got, ref)


def test_e4m3_ties_and_saturation(orc):
    assert orc.e4m3_encode(1.0625) == 0x38          # between 1 and 1.125: even (1.0)
    assert orc.e4m3_encode(1.1875) == 0x3A          # between 1.125 and 1.25: even (1.25)
    assert orc.e4m3_encode(2.0 ** -10) == 0x00      # half the smallest subnormal: to even 0
    assert orc.e4m3_encode(3 * 2.0 ** -10) == 0x02  # 1.5 quanta -> 2 quanta
    assert orc.e4m3_encode(460.0) == 0x7E
    assert orc.e4m3_encode(1e30) == 0x7E
    assert orc.e4m3_encode(-1e30) == 0xFE
    assert orc.e4m3_encode(float("inf")) == 0x7E


@pytest.mark.parametrize("amax,s", [(10.14, 32.0), (1.0, 256.0), (0.999, 256.0), (448.0, 1.0),
                                    (449.0, 0.5), (0.0, 1.0), (1e-3, 262144.0)])
def test_pow2_scale(orc, amax, s):
    assert orc.pow2_scale(amax) == s
    if amax > 0:
        assert amax * s <= 448.0 < amax * s * 2


def test_quantize_rows_and_whole(orc):
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, size=(5, 9)).astype(np.float32)
    x[3] *= 0.01
    q, inv = orc.quantize(x, "e4m3", per_row=True)
    assert q.dtype == np.uint8 and inv.shape == (5,)
    for r in range(5):
        s = orc.pow2_scale(float(np.max(np.abs(x[r]))))
        assert inv[r] == np.float32(1.0 / s)
        for c in range(9):
            assert q[r, c] == orc.e4m3_encode(float(x[r, c]) * s)
    deq = orc.e4m3_decode_array(q) * inv[:, None]
    assert np.max(np.abs(deq - x) / np.max(np.abs(x), axis=1, keepdims=True)) <= 2 ** -4
    qw, invw = orc.quantize(x, "e4m3", per_row=False)
    assert invw.shape == (1,) and invw[0] == np.float32(1.0 / orc.pow2_scale(float(np.max(np.abs(x)))))
    qb, invb = orc.quantize(x, "bf16", per_row=True)
    assert qb.dtype == np.uint16 and np.all(invb == 1.0)
    np.testing.assert_array_equal(orc.bf16_decode_array(qb),
                                  torch.from_numpy(x).to(torch.bfloat16).float().numpy())
