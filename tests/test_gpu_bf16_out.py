"""GPU parity of the bf16 output option of matmul and Linear (bf16 or e4m3
inputs, fp32 accumulation, the result -- plus the bf16 C read back when
accumulating, plus the bias -- rounded once to bf16 in the output stage).

Small-integer operands keep every fp32 partial sum exact, so the kernel's bf16
code must equal the oracle's exact result rounded to bf16 (round to nearest
even), bit for bit.  Normal operands: each element within one bf16 rounding of
the double result plus the fp32 accumulation error.  Guard columns around C
catch writes outside the output; a split over K is refused.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_16080_amd as mlk
from paper_2307_16080_amd import _lib as L
from workloads import linear_bias, matmul_inputs, random_c

from gpu_util import all_tiles, bits16, from_bf16_codes, from_e4m3_codes, dev, host, normwise, say

pytestmark = pytest.mark.gpu

RAGGED = [(1, 1, 1), (7, 13, 31), (129, 257, 100), (255, 511, 513), (300, 272, 256)]
GUARD = 3
SENTINEL = 0x7FA5  # a bf16 NaN code the kernels never write (theirs is 0x7FC0 or 0xFFC0)


def _operands(dt, A, B):
    if dt == L.MLK_BF16:
        qa, qb = oracle.bf16_encode(A), oracle.bf16_encode(B)
        return from_bf16_codes(qa), from_bf16_codes(qb), oracle.bf16_decode(qa), oracle.bf16_decode(qb)
    qa, qb = oracle.e4m3_encode(A, 1.0), oracle.e4m3_encode(B, 1.0)
    return from_e4m3_codes(qa), from_e4m3_codes(qb), oracle.e4m3_decode(qa), oracle.e4m3_decode(qb)


def _c_with_guard(codes):
    """bf16 C with ldc = N + GUARD and an extra row; the margin holds SENTINEL."""
    M, N = codes.shape
    big = np.full((M + 1, N + GUARD), SENTINEL, np.uint16)
    big[:M, :N] = codes
    t = from_bf16_codes(big)
    return t, t[:M, :N]


def _check_guard(big, M, N):
    h = bits16(big)
    assert np.all(h[:M, N:] == SENTINEL) and np.all(h[M, :] == SENTINEL), "write outside C"


def _tiles():
    """Every tile that writes a bf16 C (the register-loaded fast tiles do not)."""
    out = []
    for dt in (L.MLK_BF16, L.MLK_F8E4M3):
        # (the register-loaded fast tiles and the 32x32 MFMA tiles have no bf16 output stage)
        out += [(dt, c) for c in all_tiles(dt, L.MLK_F32) if c.stages != 1 and c.mfma != 32]
    return out


def _id(p):
    dt, c = p
    return f"{'bf16' if dt == L.MLK_BF16 else 'e4m3'}_{c.bm}x{c.bn}x{c.bk}_{c.wm}{c.wn}_s{c.stages}_m{c.mfma}"


@pytest.mark.parametrize("p", _tiles(), ids=_id)
def test_bf16_out_every_tile_exact(p):
    dt, cfg = p
    for (M, N, K) in RAGGED:
        say("bf16 out", _id(p), M, N, K)
        A, B = matmul_inputs(M, N, K, seed=M + N + K, dist="small_int")
        da, db, va, vb = _operands(dt, A, B)
        # overwrite: C starts as NaN codes that must never be read
        big, C = _c_with_guard(np.full((M, N), 0x7FC0, np.uint16))
        mlk.matmul(da, db, C, accumulate=False, cfg=cfg)
        want = oracle.bf16_encode(oracle.matmul_f64(va, vb))
        assert np.array_equal(bits16(C), want), "overwrite"
        _check_guard(big, M, N)
        # accumulate into a bf16 C of small integers
        c0 = oracle.bf16_encode(np.rint(random_c(M, N, seed=K) * 8))
        big, C = _c_with_guard(c0)
        mlk.matmul(da, db, C, accumulate=True, cfg=cfg)
        want = oracle.bf16_encode(oracle.matmul_f64(va, vb, oracle.bf16_decode(c0)))
        assert np.array_equal(bits16(C), want), "accumulate"
        _check_guard(big, M, N)
        # Linear with a bf16 output
        bias = linear_bias(N, K, "small_int")
        big, C = _c_with_guard(c0)
        mlk.matmul_bias(da, db, dev(bias), C, accumulate=True, cfg=cfg)
        want = oracle.bf16_encode(oracle.linear_f64(va, vb, bias, oracle.bf16_decode(c0)))
        assert np.array_equal(bits16(C), want), "linear"
        _check_guard(big, M, N)


@pytest.mark.parametrize("p", [q for q in _tiles() if q[0] == L.MLK_BF16], ids=_id)
def test_bf16_out_normal_within_one_rounding(p):
    dt, cfg = p
    for (M, N, K) in RAGGED[2:]:
        say("bf16 out normal", _id(p), M, N, K)
        A, B = matmul_inputs(M, N, K, seed=M + 3 * N + K, dist="normal")
        da, db, va, vb = _operands(dt, A, B)
        c0 = oracle.bf16_encode(random_c(M, N, seed=K + 1))
        bias = linear_bias(N, M, "normal")
        exact = oracle.linear_f64(va, vb, bias, oracle.bf16_decode(c0))
        mag = oracle.matmul_f64(np.abs(va), np.abs(vb)) + np.abs(bias)[None, :] + np.abs(oracle.bf16_decode(c0))
        C = from_bf16_codes(c0)
        mlk.matmul_bias(da, db, dev(bias), C, accumulate=True, cfg=cfg)
        got = oracle.bf16_decode(bits16(C))
        # one rounding to bf16 (half an ulp: 2^-9 relative) of an fp32 sum whose
        # own error stays far below 2^-16 of the magnitudes summed
        bound = 2.0 ** -8 * np.abs(exact) + 2.0 ** -16 * mag
        assert np.all(np.abs(got - exact) <= bound), float(np.max(np.abs(got - exact) / bound))
        e = normwise(got, exact)
        say("  normwise", e)
        assert e <= 2.0 ** -8


def test_bf16_out_e4m3_scaled():
    M, N, K = 257, 528, 640
    A, B = matmul_inputs(M, N, K, seed=21, dist="normal")
    qa, sa = oracle.quantize_e4m3(A)
    qb, sb = oracle.quantize_e4m3(B)
    alpha = float(np.float32(sa)) * float(np.float32(sb))
    va, vb = oracle.e4m3_decode(qa), oracle.e4m3_decode(qb)
    exact = alpha * oracle.matmul_f64(va, vb)
    mag = alpha * oracle.matmul_f64(np.abs(va), np.abs(vb))
    for cfg in [c for c in all_tiles(L.MLK_F8E4M3, L.MLK_F32) if c.stages != 1]:
        say("bf16 out e4m3 scaled", cfg)
        C = torch.empty(M, N, dtype=torch.bfloat16, device="cuda")
        mlk.matmul(from_e4m3_codes(qa), from_e4m3_codes(qb), C, accumulate=False, cfg=cfg,
                   scale_a=dev(np.array([sa], np.float32)), scale_b=dev(np.array([sb], np.float32)))
        got = oracle.bf16_decode(bits16(C))
        bound = 2.0 ** -8 * np.abs(exact) + 2.0 ** -13 * mag   # the e4m3 MFMA's own error included
        assert np.all(np.abs(got - exact) <= bound), float(np.max(np.abs(got - exact) / bound))


def test_bf16_out_refuses_split_k_and_register_loaded_tiles():
    M, N, K = 64, 64, 1024
    A = torch.zeros(M, K, dtype=torch.bfloat16, device="cuda")
    B = torch.zeros(K, N, dtype=torch.bfloat16, device="cuda")
    C = torch.zeros(M, N, dtype=torch.bfloat16, device="cuda")
    c = all_tiles(L.MLK_BF16, L.MLK_F32)[0]
    with pytest.raises(mlk.MlkError):
        mlk.matmul(A, B, C, cfg=mlk.TileConfig(c.bm, c.bn, c.bk, c.wm, c.wn, 2, 1, 0, c.stages, c.layout))
    reg = [t for t in all_tiles(L.MLK_BF16, L.MLK_F32) if t.stages == 1 or t.mfma == 32]
    assert any(t.mfma == 32 for t in reg)
    for t in reg:
        with pytest.raises(mlk.MlkError):
            mlk.matmul(A, B, C, cfg=t)
    # the default (heuristic) configuration of a small-M, deep product does not split
    mlk.matmul(A, B, C)
    assert not torch.any(C.float() != 0).item()


def test_bf16_out_headline_shape_sampled():
    """4096^3 bf16 -> bf16 Linear in the default configuration, sampled rows."""
    M = N = K = 4096
    A, B = matmul_inputs(M, N, K, seed=3, dist="normal")
    qa, qb = oracle.bf16_encode(A), oracle.bf16_encode(B)
    bias = linear_bias(N, 8, "normal")
    C = torch.empty(M, N, dtype=torch.bfloat16, device="cuda")
    mlk.matmul_bias(from_bf16_codes(qa), from_bf16_codes(qb), dev(bias), C, accumulate=False)
    got = oracle.bf16_decode(bits16(C))
    rows = np.random.default_rng(0).choice(M, 16, replace=False)
    va, vb = oracle.bf16_decode(qa)[rows], oracle.bf16_decode(qb)
    exact = oracle.linear_f64(va, vb, bias, threads=8)
    mag = oracle.matmul_f64(np.abs(va), np.abs(vb), threads=8) + np.abs(bias)[None, :]
    bound = 2.0 ** -8 * np.abs(exact) + 2.0 ** -16 * mag
    assert np.all(np.abs(got[rows] - exact) <= bound)


def test_bf16_out_k_zero():
    """K = 0 with a bf16 C: the Linear writes the bias rounded to bf16; the plain
    product leaves C (accumulate) or writes +0 (overwrite)."""
    M, N = 37, 70
    A = torch.zeros(M, 0, dtype=torch.bfloat16, device="cuda")
    B = torch.zeros(0, N, dtype=torch.bfloat16, device="cuda")
    bias = linear_bias(N, 1, "normal")
    C = from_bf16_codes(np.full((M, N), 0x7FC0, np.uint16))
    mlk.matmul_bias(A, B, dev(bias), C, accumulate=False)
    assert np.array_equal(bits16(C), oracle.bf16_encode(np.broadcast_to(bias, (M, N))))
    c0 = oracle.bf16_encode(random_c(M, N, seed=3))
    C = from_bf16_codes(c0)
    mlk.matmul(A, B, C, accumulate=True)
    assert np.array_equal(bits16(C), c0)
    mlk.matmul(A, B, C, accumulate=False)
    assert np.all(bits16(C) == 0)
