"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers and lists problem shapes.  It holds none
of the kernels' arithmetic (no product, no rounding, no quantisation), so the
oracle and the GPU library can both be fed from it without sharing code.

Generators use numpy's PCG64 (``default_rng(seed)``), drawing A then B (or x
then w) in that order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


# --------------------------------------------------------------------------- matmul

def matmul_inputs(M: int, N: int, K: int, seed: int = 0, dist: str = "uniform"):
    """A (M x K) then B (K x N), float32 unless dist == "int8".

    dist: "uniform"   uniform[-1, 1)
          "normal"    standard normal
          "int8"      integers uniform in [-128, 127] (int8)
          "small_int" integers uniform in [-8, 8] (float32; exact in bf16 and
                      e4m3, and every fp32 partial sum is exact)
          "ones"      all ones
    """
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        A = rng.uniform(-1.0, 1.0, (M, K)).astype(np.float32)
        B = rng.uniform(-1.0, 1.0, (K, N)).astype(np.float32)
    elif dist == "normal":
        A = rng.standard_normal((M, K), dtype=np.float32)
        B = rng.standard_normal((K, N), dtype=np.float32)
    elif dist == "int8":
        A = rng.integers(-128, 128, (M, K), dtype=np.int8)
        B = rng.integers(-128, 128, (K, N), dtype=np.int8)
    elif dist == "small_int":
        A = rng.integers(-8, 9, (M, K)).astype(np.float32)
        B = rng.integers(-8, 9, (K, N)).astype(np.float32)
    elif dist == "ones":
        A = np.ones((M, K), np.float32)
        B = np.ones((K, N), np.float32)
    else:
        raise ValueError(f"unknown distribution {dist!r}")
    return A, B


def random_c(M: int, N: int, seed: int, dtype=np.float32):
    """A nonzero starting C, to check that the kernels accumulate into it."""
    rng = np.random.default_rng(seed + 7919)
    if np.dtype(dtype) == np.int32:
        return rng.integers(-1000, 1000, (M, N), dtype=np.int32)
    return rng.uniform(-1.0, 1.0, (M, N)).astype(dtype)


def linear_bias(N: int, seed: int, dist: str = "normal"):
    """The bias vector of a Linear layer (N float32 values).

    dist: "normal" standard normal; "small_int" integers uniform in [-8, 8]
    (sums with small-integer products stay exact in fp32)."""
    rng = np.random.default_rng(seed + 104729)
    if dist == "small_int":
        return rng.integers(-8, 9, N).astype(np.float32)
    return rng.standard_normal(N).astype(np.float32)


# --------------------------------------------------------------------------- conv

def conv_inputs(N: int, C: int, H: int, W: int, F: int, KH: int, KW: int, seed: int = 0,
                dist: str = "normal"):
    """x (N, C, H, W) then w (F, C, KH, KW), float32."""
    rng = np.random.default_rng(seed)
    if dist == "normal":
        x = rng.standard_normal((N, C, H, W), dtype=np.float32)
        w = rng.standard_normal((F, C, KH, KW), dtype=np.float32)
    elif dist == "small_int":
        x = rng.integers(-4, 5, (N, C, H, W)).astype(np.float32)
        w = rng.integers(-4, 5, (F, C, KH, KW)).astype(np.float32)
    elif dist == "ones":
        x = np.ones((N, C, H, W), np.float32)
        w = np.ones((F, C, KH, KW), np.float32)
    else:
        raise ValueError(f"unknown distribution {dist!r}")
    return x, w


@dataclass(frozen=True)
class ConvShape:
    N: int
    C: int
    H: int
    W: int
    F: int
    KH: int
    KW: int
    stride: int
    pad: int

    def out_hw(self):
        ho = (self.H + 2 * self.pad - self.KH) // self.stride + 1
        wo = (self.W + 2 * self.pad - self.KW) // self.stride + 1
        return ho, wo

    def flops(self) -> int:
        ho, wo = self.out_hw()
        return 2 * self.N * self.F * ho * wo * self.C * self.KH * self.KW


# ResNet-18's convolution layers after the stem: (C, F, H_in, k, stride, pad, count).
RESNET18_LAYERS = [
    (64, 64, 56, 3, 1, 1, 4),
    (64, 128, 56, 3, 2, 1, 1),
    (64, 128, 56, 1, 2, 0, 1),
    (128, 128, 28, 3, 1, 1, 3),
    (128, 256, 28, 3, 2, 1, 1),
    (128, 256, 28, 1, 2, 0, 1),
    (256, 256, 14, 3, 1, 1, 3),
    (256, 512, 14, 3, 2, 1, 1),
    (256, 512, 14, 1, 2, 0, 1),
    (512, 512, 7, 3, 1, 1, 3),
]


def resnet18_conv_stack(batch: int):
    """[(ConvShape, count)] for the ten distinct layer shapes at one batch size."""
    return [(ConvShape(batch, c, h, h, f, k, k, s, p), n) for (c, f, h, k, s, p, n) in RESNET18_LAYERS]


# The paper's only measured workload: one 1280 x 1280 image, 3 output channels,
# 3 x 3 filter, no padding (Sec. 4.3).
PAPER_CONV = ConvShape(1, 1, 1280, 1280, 3, 3, 3, 1, 0)


# --------------------------------------------------------------------------- batched

def batched_shapes(count: int = 256, seed: int = 0, lo: int = 32, hi: int = 2048):
    """(M, N, K) triples, each drawn log-uniform on [lo, hi] and rounded."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), (count, 3))
    return [tuple(int(v) for v in row) for row in np.rint(np.exp(u)).astype(np.int64)]


def batched_inputs(shapes, seed: int = 1, dist: str = "normal"):
    """A_i then B_i per problem, in list order, from one generator."""
    rng = np.random.default_rng(seed)
    out = []
    for (M, N, K) in shapes:
        if dist == "normal":
            A = rng.standard_normal((M, K), dtype=np.float32)
            B = rng.standard_normal((K, N), dtype=np.float32)
        elif dist == "small_int":
            A = rng.integers(-8, 9, (M, K)).astype(np.float32)
            B = rng.integers(-8, 9, (K, N)).astype(np.float32)
        else:
            raise ValueError(dist)
        out.append((A, B))
    return out


# --------------------------------------------------------------------------- named configs

# Small case: fp32 matmul 128^3, uniform[-1, 1], C = 0.
CFG_MATMUL_F32_SMALL = dict(M=128, N=128, K=128, dist="uniform", seed=0)
# fp32 conv, N=1, C=64, 56x56, F=64, 3x3, stride 1, pad 1, normal(0, 1).
CFG_CONV_F32 = ConvShape(1, 64, 56, 56, 64, 3, 3, 1, 1)
# i8 x i8 -> i32 matmul 1024^3, integers in [-128, 127].
CFG_MATMUL_I8 = dict(M=1024, N=1024, K=1024, dist="int8", seed=0)
# bf16 / fp8 / fp32 matmul 4096^3, normal(0, 1).
CFG_MATMUL_PRECISION = dict(M=4096, N=4096, K=4096, dist="normal", seed=0)
