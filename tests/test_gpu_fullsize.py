"""Parity at the benchmark's full sizes, over every configuration the tuner can
pick, against the CPU oracle.

* bf16 and e4m3 4096^3 (C += A B, C starting nonzero): every 256 x 256
  direct-to-LDS two-stage configuration (both 8-wave layouts and the 4-wave
  one, group_m 1 and 8, XCD remap off and on, every split) is compared over
  the WHOLE of C with the double-precision product of the quantised codes, and
  bit for bit on small-integer inputs (every fp32 partial sum exact); every
  other legal configuration is compared on one row in each 128-row band of C
  (every output tile of every tile shape is sampled).
* fp32 4096^3 and int8 1024^3: every legal configuration over the whole
  output (int8 bit-exact).
* ResNet-18 convolutions at batch 32: every legal configuration of every
  layer on three sampled images, and the exhaustive-search pick over the
  whole output.
* The 256 uneven bf16 GEMMs in one persistent, graph-replayed launch: every
  legal batched configuration, every GEMM against the oracle (whole C for the
  small ones, one row per 64-row band plus the last row for the others).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_16080_amd as mlk
from paper_2307_16080_amd import _lib as L
from workloads import (batched_inputs, batched_shapes, conv_inputs, matmul_inputs, random_c,
                       resnet18_conv_stack)

from gpu_util import dev, from_bf16_codes, from_e4m3_codes, host, normwise, say

pytestmark = pytest.mark.gpu

E4M3_KERNEL_TOL = 5e-5  # the e4m3 MFMA's own rounding (see test_gpu_matmul)
N4K = 4096


def _band_rows(M, band, seed):
    """One row inside every `band`-row band of [0, M), at a varying offset, plus the last row."""
    rng = np.random.default_rng(seed)
    rows = [min(M - 1, b + int(rng.integers(0, band))) for b in range(0, M, band)] + [M - 1]
    return np.unique(np.array(rows))


def _is_full_256(c):
    return c.bm == 256 and c.bn == 256 and c.stages == 2


def _tag(c):
    return "[" + ",".join(str(v) for v in c.as_tuple()) + "]"


def _sweep_4096(kind, qa, qb, codes_ref, small_a, small_b, small_ref, run):
    """Every legal configuration of the 4096^3 product of one input type."""
    ind = L.MLK_BF16 if kind == "bf16" else L.MLK_F8E4M3
    cfgs = mlk.configs(mlk.matmul_problem(N4K, N4K, N4K, ind, L.MLK_F32, accumulate=True))
    tol = 1e-5 if kind == "bf16" else E4M3_KERNEL_TOL
    C0 = random_c(N4K, N4K, seed=11)
    C0d = dev(C0)
    ref = codes_ref + C0.astype(np.float64)
    rows = _band_rows(N4K, 128, seed=3)
    C = torch.empty(N4K, N4K, device="cuda")
    n_full = 0
    for c in cfgs:
        C.copy_(C0d)
        run(qa, qb, C, c)
        if _is_full_256(c):
            got = host(C)
            e = normwise(got, ref)
            say(kind, _tag(c), "whole C normwise", e)
            assert e <= tol, (_tag(c), e)
            # small integers: every partial sum exact, so bit-exact over all of C
            C.zero_()
            run(small_a, small_b, C, c)
            assert np.array_equal(host(C).astype(np.float64), small_ref), _tag(c)
            n_full += 1
        else:
            got = host(C)[rows]
            e = normwise(got, ref[rows])
            say(kind, _tag(c), "sampled rows normwise", e)
            assert e <= tol, (_tag(c), e)
    assert n_full >= 8, n_full  # both 8-wave layouts x group_m x remap at least


def test_bf16_4096_every_config():
    A, B = matmul_inputs(N4K, N4K, N4K, seed=0, dist="normal")
    oa, ob = oracle.bf16_encode(A), oracle.bf16_encode(B)
    say("oracle 4096^3 (bf16 codes)")
    codes_ref = oracle.matmul_f64(oracle.bf16_decode(oa), oracle.bf16_decode(ob), threads=oracle.default_threads())
    Sa, Sb = matmul_inputs(N4K, N4K, N4K, seed=1, dist="small_int")
    small_ref = oracle.matmul_f64(Sa, Sb, threads=oracle.default_threads())
    qa, qb = from_bf16_codes(oa), from_bf16_codes(ob)
    sa, sb = from_bf16_codes(oracle.bf16_encode(Sa)), from_bf16_codes(oracle.bf16_encode(Sb))
    _sweep_4096("bf16", qa, qb, codes_ref, sa, sb, small_ref,
                lambda a, b, C, c: mlk.matmul(a, b, C, cfg=c))


def test_e4m3_4096_every_config():
    A, B = matmul_inputs(N4K, N4K, N4K, seed=0, dist="normal")
    oa, osa = oracle.quantize_e4m3(A)
    ob, osb = oracle.quantize_e4m3(B)
    say("oracle 4096^3 (e4m3 codes)")
    alpha = float(np.float32(osa)) * float(np.float32(osb))
    codes_ref = alpha * oracle.matmul_f64(oracle.e4m3_decode(oa), oracle.e4m3_decode(ob),
                                          threads=oracle.default_threads())
    Sa, Sb = matmul_inputs(N4K, N4K, N4K, seed=1, dist="small_int")
    small_ref = oracle.matmul_f64(Sa, Sb, threads=oracle.default_threads())
    sa_d = dev(np.array([osa], np.float32))
    sb_d = dev(np.array([osb], np.float32))
    qa, qb = from_e4m3_codes(oa), from_e4m3_codes(ob)
    ia, ib = from_e4m3_codes(oracle.e4m3_encode(Sa, 1.0)), from_e4m3_codes(oracle.e4m3_encode(Sb, 1.0))

    def run(a, b, C, c):
        if a is qa:
            mlk.matmul(a, b, C, cfg=c, scale_a=sa_d, scale_b=sb_d)
        else:
            mlk.matmul(a, b, C, cfg=c)   # unit scales: small integers stay exact

    _sweep_4096("e4m3", qa, qb, codes_ref, ia, ib, small_ref, run)


def test_f32_4096_every_config():
    A, B = matmul_inputs(N4K, N4K, N4K, seed=0, dist="normal")
    say("oracle 4096^3 (fp32 inputs)")
    ref = oracle.matmul_f64(A, B, threads=oracle.default_threads())
    Ad, Bd = dev(A), dev(B)
    C = torch.empty(N4K, N4K, device="cuda")
    for c in mlk.configs(mlk.matmul_problem(N4K, N4K, N4K, L.MLK_F32, L.MLK_F32)):
        C.zero_()
        mlk.matmul(Ad, Bd, C, cfg=c)
        e = normwise(host(C), ref)
        say("f32", _tag(c), e)
        assert e <= 1e-5, (_tag(c), e)


def test_i8_1024_every_config_bit_exact():
    A, B = matmul_inputs(1024, 1024, 1024, seed=0, dist="int8")
    ref = oracle.matmul_i8(A, B, threads=oracle.default_threads())
    C0 = random_c(1024, 1024, seed=5, dtype=np.int32)
    want = (C0.astype(np.int64) + ref.astype(np.int64)).astype(np.int32)
    Ad, Bd, C0d = dev(A), dev(B), dev(C0)
    C = torch.empty(1024, 1024, dtype=torch.int32, device="cuda")
    cfgs = mlk.configs(mlk.matmul_problem(1024, 1024, 1024, L.MLK_I8, L.MLK_I32))
    for c in cfgs:
        C.zero_()
        mlk.matmul(Ad, Bd, C, cfg=c)
        assert np.array_equal(host(C), ref), _tag(c)
        C.copy_(C0d)
        mlk.matmul(Ad, Bd, C, cfg=c)
        assert np.array_equal(host(C), want), ("accumulate", _tag(c))
    say("i8 1024^3:", len(cfgs), "configurations bit-exact")


def test_resnet18_b32_every_config():
    sample = [0, 17, 31]
    for li, (shape, _count) in enumerate(resnet18_conv_stack(32)):
        x, w = conv_inputs(shape.N, shape.C, shape.H, shape.W, shape.F, shape.KH, shape.KW, seed=50 + li)
        ox, ow = oracle.bf16_encode(x), oracle.bf16_encode(w)
        say("layer", shape, "oracle (whole batch)")
        ref = oracle.conv2d_f64(oracle.bf16_decode(ox), oracle.bf16_decode(ow), (shape.stride,) * 2,
                                (shape.pad,) * 2, threads=oracle.default_threads())
        qx, qw = from_bf16_codes(ox), from_bf16_codes(ow)
        ho, wo = shape.out_hw()
        y = torch.empty(shape.N, shape.F, ho, wo, device="cuda")
        p = mlk.conv_problem(shape.N, shape.C, shape.H, shape.W, shape.F, shape.KH, shape.KW,
                             shape.stride, shape.pad, L.MLK_BF16, L.MLK_F32)
        cfgs = mlk.configs(p)
        for c in cfgs:
            y.zero_()
            mlk.conv2d_nchw_fchw(qx, qw, y, (shape.stride,) * 2, (shape.pad,) * 2, cfg=c)
            e = normwise(host(y[sample]), ref[sample])
            assert e <= 1e-5, (shape, _tag(c), e)
        # the configuration the exhaustive search picks (the benchmark's stack tile), whole output
        best, rep, _ = mlk.tune(p, mlk.MLK_TUNE_EXHAUSTIVE, reps=3, warmup=1)
        y.zero_()
        mlk.conv2d_nchw_fchw(qx, qw, y, (shape.stride,) * 2, (shape.pad,) * 2, cfg=best)
        e = normwise(host(y), ref)
        say("  ", len(cfgs), "configs on sampled images; tuned", _tag(best), "whole output", e)
        assert e <= 1e-5, (shape, _tag(best), e)


def test_resnet18_b1_every_config_bound():
    """Every legal configuration of every batch-1 ResNet-18 layer, bound as the
    benchmark's stack binds it (mlk.ConvCall), against the oracle on the whole
    output."""
    total = 0
    for li, (shape, _count) in enumerate(resnet18_conv_stack(1)):
        x, w = conv_inputs(shape.N, shape.C, shape.H, shape.W, shape.F, shape.KH, shape.KW, seed=70 + li)
        ox, ow = oracle.bf16_encode(x), oracle.bf16_encode(w)
        ref = oracle.conv2d_f64(oracle.bf16_decode(ox), oracle.bf16_decode(ow), (shape.stride,) * 2,
                                (shape.pad,) * 2, threads=oracle.default_threads())
        qx, qw = from_bf16_codes(ox), from_bf16_codes(ow)
        ho, wo = shape.out_hw()
        y = torch.empty(shape.N, shape.F, ho, wo, device="cuda")
        p = mlk.conv_problem(shape.N, shape.C, shape.H, shape.W, shape.F, shape.KH, shape.KW,
                             shape.stride, shape.pad, L.MLK_BF16, L.MLK_F32)
        cfgs = mlk.configs(p)
        say("layer", shape, len(cfgs), "configurations, bound")
        for c in cfgs:
            y.zero_()
            mlk.ConvCall(qx, qw, y, (shape.stride,) * 2, (shape.pad,) * 2, cfg=c)()
            e = normwise(host(y), ref)
            assert e <= 1e-5, (shape, _tag(c), e)
        total += len(cfgs)
    say("b1 stack:", total, "bound configurations")


def test_batched_256_every_config_all_gemms():
    shapes = batched_shapes(256, seed=0)
    ins = batched_inputs(shapes, seed=1)
    codes, probs, refs = [], [], []
    for (A, B), (M, N, K) in zip(ins, shapes):
        qa, qb = oracle.bf16_encode(A), oracle.bf16_encode(B)
        da, db = oracle.bf16_decode(qa), oracle.bf16_decode(qb)
        rows = np.arange(M) if M * N * K <= (1 << 24) else _band_rows(M, 64, seed=M + N + K)
        refs.append((rows, oracle.matmul_f64(da[rows], db, threads=oracle.default_threads())))
        probs.append((from_bf16_codes(qa), from_bf16_codes(qb), torch.zeros(M, N, device="cuda")))
    say("oracle rows for 256 GEMMs done;", sum(len(r) == s[0] for (r, _), s in zip(refs, shapes)), "whole")
    pb = mlk.batched_problem(shapes, L.MLK_BF16, L.MLK_F32)
    best, _, _ = mlk.tune(pb, mlk.MLK_TUNE_EXHAUSTIVE, reps=3, warmup=1)
    cfgs = mlk.configs(pb)
    assert any(c.as_tuple() == best.as_tuple() for c in cfgs)
    for c in cfgs:
        call = mlk.BatchedCall(probs, cfg=c, persistent=True, graph=True)
        for rep in range(2):
            for p in probs:
                p[2].zero_()
            call()
            torch.cuda.synchronize()
            for i, ((rows, ref), p) in enumerate(zip(refs, probs)):
                got = p[2][torch.from_numpy(rows).cuda()].cpu().numpy()
                e = normwise(got, ref)
                assert e <= 1e-5, (_tag(c), rep, i, shapes[i], e)
        say("batched", _tag(c), "all 256 GEMMs within 1e-5 on two replays")
    mlk.release()
