"""GPU parity of the Linear layer (matmul with the bias add fused into the
output stage, mlk_matmul_bias) against the oracle's Linear: the product nest
into a zeroed buffer, then the bias nest adding bias[j] to every row.

Every compiled float tile runs on ragged shapes, with small-integer operands
and bias (every fp32 partial sum exact, so the result is bit-exact) and with
normal operands (normwise error against the double result on the same
quantised values); overwrite and accumulate; split K (only one split adds the
bias); K == 0; e4m3 with scales (the bias is added after the scale).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_16080_amd as mlk
from paper_2307_16080_amd import _lib as L
from workloads import linear_bias, matmul_inputs, random_c

from gpu_util import all_tiles, dev, from_bf16_codes, from_e4m3_codes, host, normwise, say

pytestmark = pytest.mark.gpu

RAGGED = [(1, 1, 1), (7, 13, 31), (129, 257, 100), (255, 511, 513), (300, 272, 256)]
E4M3_KERNEL_TOL = 5e-5   # the e4m3 MFMA's own error, as for the plain product


def _bias(N, seed, small_int):
    return linear_bias(N, seed, "small_int" if small_int else "normal")


def _operands(dt, A, B):
    """(device A, device B, exact values of A and B) for one input type."""
    if dt == L.MLK_F32:
        return dev(A.astype(np.float32)), dev(B.astype(np.float32)), A.astype(np.float32), B.astype(np.float32)
    if dt == L.MLK_BF16:
        qa, qb = oracle.bf16_encode(A), oracle.bf16_encode(B)
        return from_bf16_codes(qa), from_bf16_codes(qb), oracle.bf16_decode(qa), oracle.bf16_decode(qb)
    qa, qb = oracle.e4m3_encode(A, 1.0), oracle.e4m3_encode(B, 1.0)
    return from_e4m3_codes(qa), from_e4m3_codes(qb), oracle.e4m3_decode(qa), oracle.e4m3_decode(qb)


def _tiles():
    out = []
    for dt in (L.MLK_F32, L.MLK_BF16, L.MLK_F8E4M3):
        out += [(dt, c) for c in all_tiles(dt, L.MLK_F32)]
    return out


def _id(p):
    dt, c = p
    return f"{ {L.MLK_F32: 'f32', L.MLK_BF16: 'bf16', L.MLK_F8E4M3: 'e4m3'}[dt] }_{c.bm}x{c.bn}x{c.bk}_{c.wm}{c.wn}_s{c.stages}"


@pytest.mark.parametrize("p", _tiles(), ids=_id)
def test_linear_every_tile_ragged(p):
    dt, cfg = p
    for (M, N, K) in RAGGED:
        say("linear", _id(p), M, N, K)
        # small integers: bit-exact, overwrite (C starts as NaN: never read) and accumulate
        A, B = matmul_inputs(M, N, K, seed=M + N + K, dist="small_int")
        da, db, va, vb = _operands(dt, A, B)
        bias = _bias(N, K, True)
        C = torch.full((M, N), float("nan"), device="cuda")
        mlk.matmul_bias(da, db, dev(bias), C, accumulate=False, cfg=cfg)
        assert np.array_equal(host(C).astype(np.float64), oracle.linear_f64(va, vb, bias)), "overwrite"
        C0 = np.rint(random_c(M, N, seed=K) * 8).astype(np.float32)
        C = dev(C0)
        mlk.matmul_bias(da, db, dev(bias), C, accumulate=True, cfg=cfg)
        assert np.array_equal(host(C).astype(np.float64), oracle.linear_f64(va, vb, bias, C0)), "accumulate"
        if dt == L.MLK_F8E4M3:
            continue   # normal-valued e4m3 runs with its scales below
        # normal operands and bias: normwise against the double result
        A, B = matmul_inputs(M, N, K, seed=M + 3 * N + K, dist="normal")
        da, db, va, vb = _operands(dt, A, B)
        bias = _bias(N, M, False)
        C0 = random_c(M, N, seed=K + 1)
        C = dev(C0)
        mlk.matmul_bias(da, db, dev(bias), C, accumulate=True, cfg=cfg)
        e = normwise(host(C), oracle.linear_f64(va, vb, bias, C0))
        say("  err", e)
        assert e <= 1e-5


@pytest.mark.parametrize("dt", [L.MLK_F32, L.MLK_BF16, L.MLK_F8E4M3], ids=["f32", "bf16", "e4m3"])
def test_linear_split_k_adds_bias_once(dt):
    M, N, K = 200, 144, 1024
    A, B = matmul_inputs(M, N, K, seed=9, dist="small_int")
    da, db, va, vb = _operands(dt, A, B)
    bias = _bias(N, 4, True)
    base = [c for c in all_tiles(dt, L.MLK_F32)]
    for c in (base[0], base[-1]):
        for sk in (2, 4):
            cfg = mlk.TileConfig(c.bm, c.bn, c.bk, c.wm, c.wn, sk, 1, 0, c.stages, c.layout)
            if not mlk.config_legal(mlk.matmul_problem(M, N, K, dt, L.MLK_F32), cfg):
                continue
            say("linear split", dt, cfg, sk)
            C = torch.full((M, N), float("nan"), device="cuda")
            mlk.matmul_bias(da, db, dev(bias), C, accumulate=False, cfg=cfg)
            assert np.array_equal(host(C).astype(np.float64), oracle.linear_f64(va, vb, bias))
            C0 = np.full((M, N), 3.0, np.float32)
            C = dev(C0)
            mlk.matmul_bias(da, db, dev(bias), C, accumulate=True, cfg=cfg)
            assert np.array_equal(host(C).astype(np.float64), oracle.linear_f64(va, vb, bias, C0))


def test_linear_k_zero_is_bias():
    M, N = 37, 70
    bias = _bias(N, 1, False)
    A = torch.zeros(M, 0, device="cuda")
    B = torch.zeros(0, N, device="cuda")
    C = torch.full((M, N), float("nan"), device="cuda")
    mlk.matmul_bias(A, B, dev(bias), C, accumulate=False)
    assert np.array_equal(host(C), np.broadcast_to(bias, (M, N)))
    C0 = random_c(M, N, seed=2)
    C = dev(C0)
    mlk.matmul_bias(A, B, dev(bias), C, accumulate=True)
    # one fp32 addition per element: the correctly rounded sum
    ref = oracle.linear_f64(np.zeros((M, 0)), np.zeros((0, N)), bias, C0).astype(np.float32)
    assert np.array_equal(host(C), ref)


def test_linear_e4m3_scaled():
    """C (+)= scale_a * scale_b * (A_q B_q) + bias on every e4m3 tile."""
    M, N, K = 257, 528, 640
    A, B = matmul_inputs(M, N, K, seed=21, dist="normal")
    qa, sa = oracle.quantize_e4m3(A)
    qb, sb = oracle.quantize_e4m3(B)
    alpha = float(np.float32(sa)) * float(np.float32(sb))
    prod = oracle.matmul_f64(oracle.e4m3_decode(qa), oracle.e4m3_decode(qb))
    bias = _bias(N, 6, False)
    C0 = random_c(M, N, seed=5)
    ref = C0.astype(np.float64) + (alpha * prod + bias.astype(np.float64)[None, :])
    for cfg in all_tiles(L.MLK_F8E4M3, L.MLK_F32):
        say("linear e4m3 scaled", cfg)
        C = dev(C0)
        mlk.matmul_bias(from_e4m3_codes(qa), from_e4m3_codes(qb), dev(bias), C, accumulate=True, cfg=cfg,
                        scale_a=dev(np.array([sa], np.float32)), scale_b=dev(np.array([sb], np.float32)))
        e = normwise(host(C), ref)
        say("  err", e)
        assert e <= E4M3_KERNEL_TOL


def test_linear_headline_shape_sampled():
    """The 4096^3 bf16 product with a bias, in the tuned/default configuration:
    sampled rows against the oracle's Linear on those rows."""
    M = N = K = 4096
    A, B = matmul_inputs(M, N, K, seed=3, dist="normal")
    qa, qb = oracle.bf16_encode(A), oracle.bf16_encode(B)
    bias = _bias(N, 8, False)
    C = torch.empty(M, N, device="cuda")
    mlk.matmul_bias(from_bf16_codes(qa), from_bf16_codes(qb), dev(bias), C, accumulate=False)
    got = host(C)
    rows = np.random.default_rng(0).choice(M, 24, replace=False)
    ref = oracle.linear_f64(oracle.bf16_decode(qa)[rows], oracle.bf16_decode(qb), bias, threads=8)
    e = normwise(got[rows], ref)
    say("4096^3 linear sampled err", e)
    assert e <= 1e-5
