"""Pins for the oracle's number formats: bf16 and OCP e4m3 encode/decode,
per-tensor scale and amax (the bf16 / fp8 extension of the paper's f32 kernels).

Fixed by: the hand-checked fixtures in tests/golden (from the format
definitions), torch's own bfloat16 / float8_e4m3fn conversions (library
routines, round-to-nearest-even), exhaustive decode/re-encode round trips,
and monotonicity.
"""
import json
import os

import numpy as np
import pytest
import torch

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_bf16_golden(orc):
    g = _load("bf16.json")
    for v, code in g["encode"]:
        assert int(orc.bf16_encode(np.array([v], np.float32))[0]) == int(code, 16), v
    for code, v in g["decode"]:
        got = orc.bf16_decode(np.array([int(code, 16)], np.uint16))[0]
        assert got == float(v)


def test_bf16_decode_all_codes_vs_torch(orc):
    codes = np.arange(65536, dtype=np.uint16)
    got = orc.bf16_decode(codes)
    want = torch.from_numpy(codes.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], want[~nan])


def test_bf16_roundtrip_all_finite_codes(orc):
    codes = np.arange(65536, dtype=np.uint16)
    vals = orc.bf16_decode(codes)
    fin = np.isfinite(vals)
    back = orc.bf16_encode(vals[fin].astype(np.float32))
    assert np.array_equal(back, codes[fin])


def test_bf16_encode_matches_torch_rne(orc):
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(200000).astype(np.float32),
        (rng.standard_normal(20000) * 1e30).astype(np.float32),
        (rng.standard_normal(20000) * 1e-39).astype(np.float32),   # subnormals
        # exact ties: a bf16 value plus half an ulp
        (np.arange(1, 4000, dtype=np.uint32) << 16 | 0x8000).view(np.float32),
        np.array([0.0, -0.0, np.inf, -np.inf, 3.4e38, -3.4e38], np.float32),
    ])
    got = orc.bf16_encode(x)
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got, want)


def test_bf16_nan(orc):
    got = orc.bf16_encode(np.array([np.nan], np.float32))[0]
    assert (got & 0x7F80) == 0x7F80 and (got & 0x7F) != 0


def test_e4m3_golden(orc):
    g = _load("e4m3_ocp.json")
    for code, v in g["decode"]:
        got = orc.e4m3_decode(np.array([int(code, 16)], np.uint8))[0]
        assert got == v and np.signbit(got) == np.signbit(v), code
    for code in g["nan_codes"]:
        assert np.isnan(orc.e4m3_decode(np.array([int(code, 16)], np.uint8))[0])
    for v, code in g["encode"]:
        assert orc.e4m3_from_float(v) == int(code, 16), v


def test_e4m3_decode_all_codes_vs_torch(orc):
    codes = np.arange(256, dtype=np.uint8)
    got = orc.e4m3_decode(codes)
    want = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], want[~nan])
    assert np.nanmax(got) == 448.0


def test_e4m3_roundtrip_all_codes(orc):
    codes = np.arange(256, dtype=np.uint8)
    vals = orc.e4m3_decode(codes)
    ok = ~np.isnan(vals)
    back = orc.e4m3_encode(vals[ok].astype(np.float32), 1.0)
    assert np.array_equal(back, codes[ok])


def test_e4m3_encode_matches_torch_inside_range(orc):
    rng = np.random.default_rng(1)
    v = np.concatenate([
        rng.uniform(-448, 448, 100000), rng.standard_normal(100000) * 0.01,
        # exact midpoints between neighbouring finite codes
        0.5 * (orc.e4m3_decode(np.arange(0, 126, dtype=np.uint8)) +
               orc.e4m3_decode(np.arange(1, 127, dtype=np.uint8))),
    ]).astype(np.float32)
    got = orc.e4m3_encode(v, 1.0)
    want = torch.from_numpy(v).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(got, want)


def test_e4m3_saturates(orc):
    v = np.array([448.0, 449.0, 464.0, 1e6, np.float32(3e38), -500.0], np.float32)
    assert list(orc.e4m3_encode(v, 1.0)) == [0x7E, 0x7E, 0x7E, 0x7E, 0x7E, 0xFE]


def test_e4m3_monotone(orc):
    v = np.linspace(-460, 460, 200001).astype(np.float32)
    dec = orc.e4m3_decode(orc.e4m3_encode(v, 1.0))
    assert np.all(np.diff(dec) >= 0)
    # nearest: the error never exceeds half the gap to the neighbouring code
    inside = np.abs(v) <= 448
    err = np.abs(dec[inside] - v[inside].astype(np.float64))
    assert np.all(err <= np.maximum(np.abs(v[inside]) * 2.0 ** -4, 2.0 ** -10) + 1e-12)


def test_scale_and_amax(orc):
    x = np.array([0.5, -3.0, 2.0, -0.0], np.float32)
    assert orc.amax(x) == 3.0
    assert orc.amax(np.zeros(0, np.float32)) == 0.0
    assert orc.e4m3_scale(448.0) == 1.0
    assert orc.e4m3_scale(0.0) == 1.0
    assert orc.e4m3_scale(3.0) == np.float32(3.0 / 448.0)
    codes, s = orc.quantize_e4m3(x)
    # the element of largest magnitude lands exactly on +-448
    assert orc.e4m3_decode(codes)[1] == -448.0
    assert s == np.float32(3.0 / 448.0)


@pytest.mark.parametrize("seed", [0, 1])
def test_quantised_values_within_half_ulp(orc, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(50000).astype(np.float32)
    codes, s = orc.quantize_e4m3(x)
    q = orc.e4m3_decode(codes) * s
    rel = np.abs(q - x) / np.maximum(np.abs(x), 1e-30)
    normal = np.abs(x) / s >= 2.0 ** -6
    assert np.max(rel[normal]) <= 2.0 ** -4 * (1 + 1e-6)
    b = orc.bf16_decode(orc.bf16_encode(x))
    assert np.max(np.abs(b - x) / np.abs(x)) <= 2.0 ** -8
