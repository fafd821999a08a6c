"""GPU parity of the matmul kernels (C ABI through the binding) against the
CPU oracle: fp32 (normwise <= 1e-5), int8 -> int32 (bit-exact), bf16 and OCP
e4m3 (kernel error against the double result on the quantised values, and
bit-exact on small-integer inputs, where every fp32 partial sum is exact).
Shapes span several tiles and ragged tails; every compiled tile kernel runs.
Guard bands around C catch writes outside the output.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_16080_amd as mlk
from paper_2307_16080_amd import _lib as L
from workloads import matmul_inputs, random_c

from gpu_util import (all_tiles, bits16, bits8, dev, from_bf16_codes, from_e4m3_codes, host,
                      normwise, say)

pytestmark = pytest.mark.gpu

RAGGED = [(1, 1, 1), (7, 13, 31), (33, 65, 17), (129, 257, 100), (300, 200, 129), (64, 64, 64),
          (255, 511, 513)]
GUARD = 3  # extra columns of sentinel on each row of C
# The e4m3 MFMA (16x16x128 f8f6f4) forms each 128-term dot product with about
# 16 significant bits before adding it to the fp32 accumulator: measured
# normwise error 1.5e-5 against the double result on the same codes,
# independent of K (32 .. 4096).  The stated bound keeps a 3x margin; it is
# three orders of magnitude below the e4m3 quantisation error itself (2^-4).
E4M3_KERNEL_TOL = 5e-5


def _with_guard(C0, dtype):
    """C stored with ldc = N + GUARD; the extra columns hold a sentinel."""
    M, N = C0.shape
    big = torch.full((M + 1, N + GUARD), -777, dtype=dtype, device="cuda")
    big[:M, :N] = dev(C0)
    return big, big[:M, :N]


def _check_guard(big, M, N):
    h = host(big)
    assert np.all(h[:M, N:] == -777) and np.all(h[M, :] == -777), "write outside C"


# ----------------------------------------------------------------------- fp32

def test_f32_config0_128():
    A, B = matmul_inputs(128, 128, 128, seed=0, dist="uniform")
    ref = oracle.matmul_f64(A, B)
    C = torch.zeros(128, 128, dtype=torch.float32, device="cuda")
    mlk.matmul(dev(A), dev(B), C)
    err = normwise(host(C), ref)
    say("f32 128^3 normwise", err)
    assert err <= 1e-5


@pytest.mark.parametrize("cfg", all_tiles(L.MLK_F32, L.MLK_F32), ids=lambda c: f"{c.bm}x{c.bn}x{c.bk}_{c.wm}{c.wn}_s{c.stages}_m{c.mfma}")
def test_f32_every_tile_ragged(cfg):
    for (M, N, K) in RAGGED:
        say("f32", cfg, M, N, K)
        A, B = matmul_inputs(M, N, K, seed=M + N + K, dist="uniform")
        C0 = random_c(M, N, seed=K)
        ref = oracle.matmul_f64(A, B, C0)
        big, C = _with_guard(C0, torch.float32)
        mlk.matmul(dev(A), dev(B), C, cfg=cfg)
        assert normwise(host(C), ref) <= 1e-5
        _check_guard(big, M, N)
        # small integers: exact
        A, B = matmul_inputs(M, N, K, seed=1, dist="small_int")
        C = torch.zeros(M, N, dtype=torch.float32, device="cuda")
        mlk.matmul(dev(A), dev(B), C, cfg=cfg)
        assert np.array_equal(host(C).astype(np.float64), oracle.matmul_f64(A, B))


def test_f32_overwrite_split_k_and_unaligned():
    M, N, K = 200, 150, 1000
    A, B = matmul_inputs(M, N, K, seed=5, dist="small_int")
    ref = oracle.matmul_f64(A, B)
    for sk in (1, 2, 4, 8):
        cfg = mlk.TileConfig(64, 64, 16, 2, 2, sk, 1, 0)
        C = torch.full((M, N), float("nan"), device="cuda")
        mlk.matmul(dev(A), dev(B), C, accumulate=False, cfg=cfg)
        assert np.array_equal(host(C).astype(np.float64), ref), sk
    # leading dimensions that are not multiples of 16 bytes: element loads
    Abig = dev(np.pad(A, ((0, 0), (0, 1))))
    Bbig = dev(np.pad(B, ((0, 0), (0, 3))))
    C = torch.zeros(M, N, device="cuda")
    mlk.matmul(Abig[:, :K], Bbig[:, :N], C)
    assert np.array_equal(host(C).astype(np.float64), ref)


def test_empty_and_k0():
    C = torch.full((4, 5), 3.0, device="cuda")
    A = torch.zeros(4, 0, device="cuda")
    B = torch.zeros(0, 5, device="cuda")
    mlk.matmul(A, B, C)                       # K = 0, accumulate: unchanged
    assert np.all(host(C) == 3.0)
    mlk.matmul(A, B, C, accumulate=False)     # K = 0, overwrite: zeros
    assert np.all(host(C) == 0.0)
    E = torch.zeros(0, 5, device="cuda")
    mlk.matmul(torch.zeros(0, 7, device="cuda"), torch.zeros(7, 5, device="cuda"), E)


# ----------------------------------------------------------------------- int8

def test_i8_1024_bit_exact():
    A, B = matmul_inputs(1024, 1024, 1024, seed=0, dist="int8")
    ref = oracle.matmul_i8(A, B, threads=oracle.default_threads())
    C = torch.zeros(1024, 1024, dtype=torch.int32, device="cuda")
    mlk.matmul(dev(A), dev(B), C)
    assert np.array_equal(host(C), ref)


@pytest.mark.parametrize("cfg", all_tiles(L.MLK_I8, L.MLK_I32), ids=lambda c: f"{c.bm}x{c.bn}x{c.bk}_{c.wm}{c.wn}_s{c.stages}_m{c.mfma}")
def test_i8_every_tile_ragged(cfg):
    for (M, N, K) in RAGGED:
        say("i8", cfg, M, N, K)
        A, B = matmul_inputs(M, N, K, seed=M * 3 + K, dist="int8")
        C0 = random_c(M, N, seed=N, dtype=np.int32)
        big, C = _with_guard(C0, torch.int32)
        mlk.matmul(dev(A), dev(B), C, cfg=cfg)
        assert np.array_equal(host(C), oracle.matmul_i8(A, B, C0))
        _check_guard(big, M, N)


def test_i8_split_k_and_wraparound():
    M, N, K = 96, 80, 4096
    A = np.full((M, K), -128, np.int8)
    B = np.full((K, N), -128, np.int8)
    C0 = np.full((M, N), 2**31 - 1, np.int32)   # 2^31 - 1 + 4096 * 16384 wraps
    for sk in (1, 4):
        C = dev(C0)
        mlk.matmul(dev(A), dev(B), C, cfg=mlk.TileConfig(64, 64, 64, 2, 2, sk, 1, 0))
        assert np.array_equal(host(C), oracle.matmul_i8(A, B, C0)), sk
        # the direct-to-LDS int8 tile: int32 atomics under split K wrap the same way
        C = dev(C0)
        mlk.matmul(dev(A), dev(B), C, cfg=mlk.TileConfig(64, 64, 128, 2, 2, sk, 1, 0, 3, 0))
        assert np.array_equal(host(C), oracle.matmul_i8(A, B, C0)), ("direct", sk)


# ----------------------------------------------------------------------- quantisation

@pytest.mark.parametrize("n", [1, 15, 16, 17, 1000, 65537, 1 << 20])
def test_quantize_bit_exact(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n).astype(np.float32)
    x[: min(n, 4)] *= 1e3
    xd = dev(x)
    q, _ = mlk.quantize(xd, "bf16")
    assert np.array_equal(bits16(q), oracle.bf16_encode(x))
    q8, s = mlk.quantize(xd, "e4m3")
    codes, scale = oracle.quantize_e4m3(x)
    assert host(s)[0] == np.float32(scale)
    assert np.array_equal(bits8(q8), codes)


def test_quantize_special_values():
    x = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 3.4e38, -1e-45, 1e-40, 448.0, -500.0] * 2,
                 np.float32)
    q, _ = mlk.quantize(dev(x), "bf16")
    assert np.array_equal(bits16(q), oracle.bf16_encode(x))
    finite = x[np.isfinite(x)].copy()
    q8, s = mlk.quantize(dev(finite), "e4m3")
    codes, scale = oracle.quantize_e4m3(finite)
    assert host(s)[0] == np.float32(scale) and np.array_equal(bits8(q8), codes)
    # all-zero input: scale 1
    q8, s = mlk.quantize(torch.zeros(33, device="cuda"), "e4m3")
    assert host(s)[0] == 1.0 and np.all(bits8(q8) == 0)
    # unaligned view exercises the scalar path
    base = dev(np.random.default_rng(0).standard_normal(1001).astype(np.float32))
    view = base[1:]
    q8, s = mlk.quantize(view.contiguous() if not view.is_contiguous() else view, "e4m3")
    codes, scale = oracle.quantize_e4m3(host(base)[1:])
    assert host(s)[0] == np.float32(scale) and np.array_equal(bits8(q8), codes)


@pytest.mark.parametrize("scale", [0.37, 1.0, 3.1e-5, 2.0 ** -20])
def test_quantize_e4m3_rounding_steps(scale):
    """Inputs within a few fp32 ulps of every e4m3 rounding step (after
    division by the scale), of the subnormal range and of saturation, both
    signs, in the vector (16 per thread) and the scalar kernels: codes and
    scale equal the oracle's bit for bit."""
    vals = oracle.e4m3_decode(np.arange(0, 127, dtype=np.uint8)).astype(np.float64)
    steps = np.concatenate([(vals[:-1] + vals[1:]) / 2, vals, [448.0, 464.0, 2.0 ** -6, 2.0 ** -9]])
    x = (steps * scale).astype(np.float32)
    around = [x]
    up, dn = x.copy(), x.copy()
    for _ in range(8):
        up = np.nextafter(up, np.float32(np.inf))
        dn = np.nextafter(dn, np.float32(0))
        around += [up.copy(), dn.copy()]
    x = np.concatenate(around)
    x = np.concatenate([x, -x, [np.float32(448.0 * scale)]]).astype(np.float32)
    x = x[np.abs(x) <= np.float32(448.0 * scale)]          # keep amax = 448 * scale
    for data in (x, np.concatenate([x, x[:7]])):             # length 16k and 16k + 7
        codes, sc = oracle.quantize_e4m3(data)
        q8, s = mlk.quantize(dev(data), "e4m3")
        assert host(s)[0] == np.float32(sc)
        assert np.array_equal(bits8(q8), codes)
    base = dev(np.concatenate([[0.0], x]).astype(np.float32))  # unaligned view: scalar kernel
    q8, s = mlk.quantize(base[1:], "e4m3")
    codes, sc = oracle.quantize_e4m3(x)
    assert np.array_equal(bits8(q8), codes)


def test_quantize_e4m3_dense_sweep_unit_scale():
    """With amax = 448 the scale is exactly 1 and each code is the e4m3 encoding
    of the input itself: a sweep over both signs, every exponent up to 448,
    the top seven fraction bits and six low-bit patterns (ties, one either
    side, all ones), through the vector kernel and its packed-conversion path,
    equals the oracle's codes bit for bit."""
    hi = np.arange(2 * 136 * 128, dtype=np.uint32)
    sign, rest = hi // (136 * 128), hi % (136 * 128)
    exp, top = rest // 128, rest % 128
    base = (sign << 31) | (exp << 23) | (top << 16)
    bits = np.concatenate([base | low for low in (0x0000, 0x0001, 0x7FFF, 0x8000, 0x8001, 0xFFFF)])
    x = bits.astype(np.uint32).view(np.float32)
    x = x[np.abs(x) <= np.float32(448.0)]
    x = np.concatenate([x, [np.float32(448.0)]]).astype(np.float32)
    codes, sc = oracle.quantize_e4m3(x)
    assert np.float32(sc) == np.float32(1.0)
    q8, s = mlk.quantize(dev(x), "e4m3")
    assert host(s)[0] == np.float32(1.0)
    assert np.array_equal(bits8(q8), codes)


def test_quantize_e4m3_calls_in_sequence():
    """e4m3 quantisation runs in one pass when the input fits the registers of a
    resident grid (a grid-wide barrier whose device arrival counter only grows
    from launch to launch) and in two passes beyond that.  Sizes in sequence,
    twice over, with other library work between them: every call's codes and
    scale equal the oracle's bit for bit."""
    sizes = [1 << 20, 5, 3 << 20, 65537, 1 << 22, 3]
    rng = np.random.default_rng(17)
    xs = [(rng.standard_normal(n) * rng.uniform(0.01, 100)).astype(np.float32) for n in sizes]
    refs = [oracle.quantize_e4m3(x) for x in xs]
    for rep in range(2):
        for x, (codes, sc) in zip(xs, refs):
            q8, s = mlk.quantize(dev(x), "e4m3")
            mlk.quantize(dev(x), "bf16")                 # other scratch-free work between calls
            assert host(s)[0] == np.float32(sc), (rep, x.size)
            assert np.array_equal(bits8(q8), codes), (rep, x.size)


def test_quantize_e4m3_wait_fallback(monkeypatch):
    """The one-pass kernel's waits are bounded; a workgroup that stops waiting
    scans the whole input for the maximum itself.  With the bound forced to a
    single round of polls from the host (MLK_QUANT_WAIT_POLLS=0), most
    workgroups take that path, and every call still gives the oracle's codes
    and scale; the next calls, with the default bound, are exact too (the
    exchange words are consistent after a fallback)."""
    rng = np.random.default_rng(23)
    xs = [(rng.standard_normal(n) * 3).astype(np.float32) for n in (1 << 20, 1 << 22, 1001)]
    refs = [oracle.quantize_e4m3(x) for x in xs]
    monkeypatch.setenv("MLK_QUANT_WAIT_POLLS", "0")
    for x, (codes, sc) in zip(xs, refs):
        q8, s = mlk.quantize(dev(x), "e4m3")
        assert host(s)[0] == np.float32(sc) and np.array_equal(bits8(q8), codes), x.size
    monkeypatch.delenv("MLK_QUANT_WAIT_POLLS")
    for x, (codes, sc) in zip(xs, refs):
        q8, s = mlk.quantize(dev(x), "e4m3")
        assert host(s)[0] == np.float32(sc) and np.array_equal(bits8(q8), codes), x.size


@pytest.mark.parametrize("n", [1001, 1 << 20, (1 << 24) + 4])
def test_quantize_e4m3_subnormal_inputs(n):
    """Every input an fp32 subnormal: the scale amax / 448 is subnormal too
    and 1 / scale overflows, so the multiply-by-reciprocal encoder is off and
    every value takes the exact per-value division (in the one-pass kernel,
    every register group through its second loop; in the two-pass one past
    the resident grid).  Codes and scale equal the oracle's bit for bit."""
    x = (np.random.default_rng(n % 997).standard_normal(n) * 1e-41).astype(np.float32)
    assert np.all(np.abs(x) < np.finfo(np.float32).tiny)
    codes, sc = oracle.quantize_e4m3(x)
    with np.errstate(over="ignore"):
        assert not np.isfinite(np.float32(1.0) / np.float32(sc))
    q8, s = mlk.quantize(dev(x), "e4m3")
    assert host(s)[0] == np.float32(sc)
    assert np.array_equal(bits8(q8), codes)


@pytest.mark.parametrize("n", [1 << 24, (1 << 24) + 4, (1 << 24) + 4096 * 4 + 3])
def test_quantize_e4m3_at_and_past_the_resident_grid(n):
    """The benchmark's 16.8 M elements (one pass, every resident workgroup) and
    sizes just past what the resident grid holds (two passes): the scale equals
    amax / 448 exactly and the codes equal the oracle's on the first and last
    4096 elements and on a million sampled ones."""
    x = np.random.default_rng(n % 1000).standard_normal(n).astype(np.float32)
    x[n // 3] = np.float32(-7.5)                     # a known maximum |x|
    q8, s = mlk.quantize(dev(x), "e4m3")
    sc = oracle.e4m3_scale(oracle.amax(x))
    assert host(s)[0] == np.float32(sc)
    got = bits8(q8)
    idx = np.concatenate([np.arange(4096), np.arange(n - 4096, n),
                          np.random.default_rng(3).integers(0, n, 1 << 20)])
    assert np.array_equal(got[idx], oracle.e4m3_encode(x[idx], sc))


# ----------------------------------------------------------------------- bf16 / e4m3

BF16_TILES = all_tiles(L.MLK_BF16, L.MLK_F32)
# shapes the direct-to-LDS kernels accept (K % 64 == 0, N % 8 == 0) with ragged M and N tiles
ALIGNED = [(1, 8, 64), (100, 136, 192), (257, 520, 640), (300, 264, 128), (512, 512, 1024), (33, 1000, 64)]


@pytest.mark.parametrize("cfg", [c for c in BF16_TILES if c.stages >= 2], ids=lambda c: f"{c.bm}x{c.bn}x{c.bk}_{c.wm}{c.wn}_s{c.stages}_m{c.mfma}")
def test_bf16_direct_to_lds_tiles(cfg):
    for (M, N, K) in ALIGNED:
        say("bf16 direct", cfg, M, N, K)
        A, B = matmul_inputs(M, N, K, seed=M + 3 * N + K, dist="normal")
        qa, qb = oracle.bf16_encode(A), oracle.bf16_encode(B)
        C0 = random_c(M, N, seed=K)
        ref = oracle.matmul_f64(oracle.bf16_decode(qa), oracle.bf16_decode(qb), C0)
        big, C = _with_guard(C0, torch.float32)
        mlk.matmul(from_bf16_codes(qa), from_bf16_codes(qb), C, cfg=cfg)
        e = normwise(host(C), ref)
        say("  kernel err", e)
        assert e <= 1e-5
        _check_guard(big, M, N)
        A, B = matmul_inputs(M, N, K, seed=4, dist="small_int")
        for acc in (True, False):
            C = torch.full((M, N), float("nan"), device="cuda") if not acc else torch.zeros(M, N, device="cuda")
            mlk.matmul(from_bf16_codes(oracle.bf16_encode(A)), from_bf16_codes(oracle.bf16_encode(B)), C,
                       cfg=cfg, accumulate=acc)
            assert np.array_equal(host(C).astype(np.float64), oracle.matmul_f64(A, B)), acc
    # ragged shapes and unaligned operands: packed into zero-padded copies first
    for (M, N, K) in RAGGED:
        say("bf16 direct ragged", cfg, M, N, K)
        A, B = matmul_inputs(M, N, K, seed=M + 5 * N + K, dist="normal")
        qa, qb = oracle.bf16_encode(A), oracle.bf16_encode(B)
        C0 = random_c(M, N, seed=K + 1)
        ref = oracle.matmul_f64(oracle.bf16_decode(qa), oracle.bf16_decode(qb), C0)
        big, C = _with_guard(C0, torch.float32)
        mlk.matmul(from_bf16_codes(qa), from_bf16_codes(qb), C, cfg=cfg)
        assert normwise(host(C), ref) <= 1e-5
        _check_guard(big, M, N)
        A, B = matmul_inputs(M, N, K, seed=3, dist="small_int")
        C = torch.zeros(M, N, device="cuda")
        mlk.matmul(from_bf16_codes(oracle.bf16_encode(A)), from_bf16_codes(oracle.bf16_encode(B)), C, cfg=cfg)
        assert np.array_equal(host(C).astype(np.float64), oracle.matmul_f64(A, B))
    # an operand view whose rows start 2 bytes past 16-byte alignment
    A, B = matmul_inputs(64, 72, 64, seed=9, dist="small_int")
    wide = torch.zeros(64, 65, dtype=torch.bfloat16, device="cuda")
    wide[:, 1:] = from_bf16_codes(oracle.bf16_encode(A))
    C = torch.zeros(64, 72, device="cuda")
    mlk.matmul(wide[:, 1:], from_bf16_codes(oracle.bf16_encode(B)), C, cfg=cfg)
    assert np.array_equal(host(C).astype(np.float64), oracle.matmul_f64(A, B))


@pytest.mark.parametrize("cfg", [c for c in BF16_TILES if c.stages < 2], ids=lambda c: f"{c.bm}x{c.bn}x{c.bk}_{c.wm}{c.wn}_s{c.stages}_m{c.mfma}")
def test_bf16_every_tile_ragged(cfg):
    for (M, N, K) in RAGGED:
        say("bf16", cfg, M, N, K)
        A, B = matmul_inputs(M, N, K, seed=M + 2 * N + K, dist="normal")
        qa, qb = oracle.bf16_encode(A), oracle.bf16_encode(B)
        C0 = random_c(M, N, seed=K)
        ref = oracle.matmul_f64(oracle.bf16_decode(qa), oracle.bf16_decode(qb), C0)
        big, C = _with_guard(C0, torch.float32)
        mlk.matmul(from_bf16_codes(qa), from_bf16_codes(qb), C, cfg=cfg)
        e = normwise(host(C), ref)
        say("  bf16 kernel err", e)
        assert e <= 1e-5
        _check_guard(big, M, N)
        A, B = matmul_inputs(M, N, K, seed=2, dist="small_int")
        C = torch.zeros(M, N, device="cuda")
        mlk.matmul(from_bf16_codes(oracle.bf16_encode(A)), from_bf16_codes(oracle.bf16_encode(B)), C,
                   cfg=cfg)
        assert np.array_equal(host(C).astype(np.float64), oracle.matmul_f64(A, B))


E4M3_TILES = all_tiles(L.MLK_F8E4M3, L.MLK_F32)
ALIGNED8 = [(1, 16, 128), (100, 144, 256), (257, 528, 640), (300, 272, 128), (512, 512, 1024), (33, 1008, 128)]


@pytest.mark.parametrize("cfg", [c for c in E4M3_TILES if c.stages >= 2], ids=lambda c: f"{c.bm}x{c.bn}x{c.bk}_{c.wm}{c.wn}_s{c.stages}_m{c.mfma}")
def test_e4m3_direct_to_lds_tiles(cfg):
    for (M, N, K) in ALIGNED8:
        say("e4m3 direct", cfg, M, N, K)
        A, B = matmul_inputs(M, N, K, seed=M + 7 * N + K, dist="normal")
        qa, sa = oracle.quantize_e4m3(A)
        qb, sb = oracle.quantize_e4m3(B)
        C0 = random_c(M, N, seed=K)
        prod = oracle.matmul_f64(oracle.e4m3_decode(qa), oracle.e4m3_decode(qb))
        ref = C0.astype(np.float64) + (float(np.float32(sa)) * float(np.float32(sb))) * prod
        big, C = _with_guard(C0, torch.float32)
        mlk.matmul(from_e4m3_codes(qa), from_e4m3_codes(qb), C, cfg=cfg,
                   scale_a=dev(np.array([sa], np.float32)), scale_b=dev(np.array([sb], np.float32)))
        e = normwise(host(C), ref)
        say("  kernel err", e)
        assert e <= E4M3_KERNEL_TOL
        _check_guard(big, M, N)
        A, B = matmul_inputs(M, N, K, seed=5, dist="small_int")
        C = torch.zeros(M, N, device="cuda")
        mlk.matmul(from_e4m3_codes(oracle.e4m3_encode(A, 1.0)), from_e4m3_codes(oracle.e4m3_encode(B, 1.0)),
                   C, cfg=cfg)
        assert np.array_equal(host(C).astype(np.float64), oracle.matmul_f64(A, B))
    # ragged shapes (packed into zero-padded copies first)
    for (M, N, K) in RAGGED:
        say("e4m3 direct ragged", cfg, M, N, K)
        A, B = matmul_inputs(M, N, K, seed=6, dist="small_int")
        big, C = _with_guard(np.zeros((M, N), np.float32), torch.float32)
        mlk.matmul(from_e4m3_codes(oracle.e4m3_encode(A, 1.0)), from_e4m3_codes(oracle.e4m3_encode(B, 1.0)),
                   C, cfg=cfg)
        assert np.array_equal(host(C).astype(np.float64), oracle.matmul_f64(A, B))
        _check_guard(big, M, N)


def test_e4m3_direct_scaled_accumulate_extremes():
    """C += alpha * (A_q B_q) when C / alpha is not representable: alpha outside
    [2^-60, 2^60], or a C so large that C / alpha overflows in one wave's tile."""
    cfg = next(c for c in E4M3_TILES if c.stages >= 2 and c.bm == 256 and c.bn == 256 and c.wm * c.wn == 8)
    M, N, K = 300, 272, 256
    A, B = matmul_inputs(M, N, K, seed=11, dist="normal")
    qa, _ = oracle.quantize_e4m3(A)
    qb, _ = oracle.quantize_e4m3(B)
    prod = oracle.matmul_f64(oracle.e4m3_decode(qa), oracle.e4m3_decode(qb))
    mag = oracle.matmul_f64(np.abs(oracle.e4m3_decode(qa)), np.abs(oracle.e4m3_decode(qb)))
    for sa, sb, big_c in ((2.0 ** -35, 2.0 ** -36, 0.0), (2.0 ** -25, 2.0 ** -25, 3e38), (3.0, 0.25, 0.0)):
        say("e4m3 extremes", sa, sb, big_c)
        C0 = random_c(M, N, seed=3)
        if big_c:
            C0[5, 7] = big_c          # C / alpha overflows for this element's wave
            C0[290, 260] = -big_c
        ref = C0.astype(np.float64) + (sa * sb) * prod
        C = dev(C0)
        mlk.matmul(from_e4m3_codes(qa), from_e4m3_codes(qb), C, cfg=cfg,
                   scale_a=dev(np.array([sa], np.float32)), scale_b=dev(np.array([sb], np.float32)))
        got = host(C).astype(np.float64)
        assert np.all(np.isfinite(got))
        # componentwise: the accumulator starts from C / alpha and each 128-deep
        # MFMA step rounds the running sum (measured up to 6 * 2^-24 * |C| for
        # two steps), plus the MFMA's own error on the products
        bound = 2.0 ** -20 * np.abs(C0) + 2.0 ** -14 * (sa * sb) * mag + 1e-45
        assert np.all(np.abs(got - ref) <= bound), float(np.max(np.abs(got - ref) / bound))


@pytest.mark.parametrize("cfg", [c for c in E4M3_TILES if c.stages < 2], ids=lambda c: f"{c.bm}x{c.bn}x{c.bk}_{c.wm}{c.wn}_s{c.stages}_m{c.mfma}")
def test_e4m3_every_tile_ragged(cfg):
    for (M, N, K) in RAGGED:
        say("e4m3", cfg, M, N, K)
        A, B = matmul_inputs(M, N, K, seed=M + 5 * N + K, dist="normal")
        qa, sa = oracle.quantize_e4m3(A)
        qb, sb = oracle.quantize_e4m3(B)
        C0 = random_c(M, N, seed=K)
        prod = oracle.matmul_f64(oracle.e4m3_decode(qa), oracle.e4m3_decode(qb))
        ref = C0.astype(np.float64) + (float(np.float32(sa)) * float(np.float32(sb))) * prod
        big, C = _with_guard(C0, torch.float32)
        mlk.matmul(from_e4m3_codes(qa), from_e4m3_codes(qb), C, cfg=cfg,
                   scale_a=dev(np.array([sa], np.float32)), scale_b=dev(np.array([sb], np.float32)))
        e = normwise(host(C), ref)
        say("  e4m3 kernel err", e)
        assert e <= E4M3_KERNEL_TOL
        _check_guard(big, M, N)
        # small integers, unit scales: exact
        A, B = matmul_inputs(M, N, K, seed=3, dist="small_int")
        C = torch.zeros(M, N, device="cuda")
        mlk.matmul(from_e4m3_codes(oracle.e4m3_encode(A, 1.0)),
                   from_e4m3_codes(oracle.e4m3_encode(B, 1.0)), C, cfg=cfg)
        assert np.array_equal(host(C).astype(np.float64), oracle.matmul_f64(A, B))


def _rows_ref(decode, qa, qb, rows):
    return oracle.matmul_f64(decode(qa[rows]), decode(qb), threads=oracle.default_threads())


def test_precision_4096_sampled_rows():
    """The 4096^3 workload in the launch configuration the benchmark uses
    (default resolution), checked on sampled rows against the oracle."""
    M = N = K = 4096
    A, B = matmul_inputs(M, N, K, seed=0, dist="normal")
    rows = np.random.default_rng(7).choice(M, 12, replace=False)
    rows.sort()
    Ad, Bd = dev(A), dev(B)
    exact = oracle.matmul_f64(A[rows], B, threads=oracle.default_threads())
    # bf16: quantise on the GPU (bit-exact vs the oracle), multiply
    qa, _ = mlk.quantize(Ad, "bf16")
    qb, _ = mlk.quantize(Bd, "bf16")
    oa, ob = oracle.bf16_encode(A), oracle.bf16_encode(B)
    assert np.array_equal(bits16(qa), oa) and np.array_equal(bits16(qb), ob)
    C = torch.zeros(M, N, device="cuda")
    mlk.matmul(qa, qb, C)
    got = host(C)[rows]
    e_kernel = normwise(got, _rows_ref(oracle.bf16_decode, oa, ob, rows))
    e_total = normwise(got, exact)
    say("bf16 4096 kernel err", e_kernel, "end-to-end", e_total)
    assert e_kernel <= 1e-5 and e_total <= 1e-2
    # e4m3
    qa8, sa = mlk.quantize(Ad, "e4m3")
    qb8, sb = mlk.quantize(Bd, "e4m3")
    oa8, osa = oracle.quantize_e4m3(A)
    ob8, osb = oracle.quantize_e4m3(B)
    assert np.array_equal(bits8(qa8), oa8) and np.array_equal(bits8(qb8), ob8)
    C = torch.zeros(M, N, device="cuda")
    mlk.matmul(qa8, qb8, C, scale_a=sa, scale_b=sb)
    got = host(C)[rows]
    ref = (float(np.float32(osa)) * float(np.float32(osb))) * _rows_ref(oracle.e4m3_decode, oa8, ob8, rows)
    e_kernel = normwise(got, ref)
    e_total = normwise(got, exact)
    say("e4m3 4096 kernel err", e_kernel, "end-to-end", e_total)
    assert e_kernel <= E4M3_KERNEL_TOL and e_total <= 0.1
    # fp32 plain kernel
    C = torch.zeros(M, N, device="cuda")
    mlk.matmul(Ad, Bd, C)
    e = normwise(host(C)[rows], exact)
    say("f32 4096 err", e)
    assert e <= 1e-5


# ----------------------------------------------------------------------- direct-layout edge

@pytest.mark.parametrize("kind", ["bf16", "e4m3", "i8"])
def test_direct_tiles_last_k_row_with_unaligned_n(kind):
    """K a whole number of stages and N not a multiple of the 16-byte chunk:
    the last K row of B ends inside a chunk.  Every direct-to-LDS tile, with B
    as a plain (M, N) tensor and as a view whose 16-byte-aligned row pitch
    exceeds N, must still sum that row's products (bit-exact on small
    integers; the oracle in double elsewhere)."""
    din = {"bf16": L.MLK_BF16, "e4m3": L.MLK_F8E4M3, "i8": L.MLK_I8}[kind]
    dout = L.MLK_I32 if kind == "i8" else L.MLK_F32
    tiles = [c for c in all_tiles(din, dout) if c.stages >= 2]
    assert tiles
    for (M, N, K) in ((519, 625, 64), (37, 13, 128), (130, 255, 256)):
        Kk = K if kind == "bf16" else 2 * K          # a whole number of 128-deep stages for 1-byte inputs
        P = (N + 15) // 16 * 16 + 16                 # a 16-byte-aligned row pitch beyond N
        if kind == "i8":
            A, B = matmul_inputs(M, N, Kk, seed=M + N, dist="int8")
            ref = oracle.matmul_i8(A, B)
            a, b_full = dev(A), torch.zeros(Kk, P, dtype=torch.int8, device="cuda")
            b_full[:, :N] = dev(B)
            cdt = torch.int32
        else:
            A, B = matmul_inputs(M, N, Kk, seed=M + N, dist="small_int")
            ref = oracle.matmul_f64(A, B)
            enc = (lambda x: from_bf16_codes(oracle.bf16_encode(x))) if kind == "bf16" else \
                  (lambda x: from_e4m3_codes(oracle.e4m3_encode(x, 1.0)))
            a = enc(A)
            Bw = np.zeros((Kk, P), np.float32)
            Bw[:, :N] = B
            b_full = enc(Bw)
            cdt = torch.float32
        for b in (b_full[:, :N].contiguous(), b_full[:, :N]):   # plain, and a pitched view
            for c in tiles:
                C = torch.zeros(M, N, dtype=cdt, device="cuda")
                mlk.matmul(a, b, C, cfg=c)
                got = host(C)
                assert np.array_equal(got.astype(ref.dtype), ref), (kind, (M, N, Kk), c, b.stride())
