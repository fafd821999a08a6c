"""mlk_matmul_noalloc (the entry point for callers that cannot allocate) against
mlk_matmul on the same inputs and tile: its packed operand copies live in the
library's fixed per-device array instead of the scratch buffer, so the two
must agree bit for bit, and both must match the oracle.  Two calls in a row,
the second on a smaller problem, reuse the array; a shape whose packed copies
exceed the array is refused before anything is enqueued."""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_16080_amd as mlk
from paper_2307_16080_amd import _lib as L
from workloads import matmul_inputs, random_c

from gpu_util import dev, from_bf16_codes, from_e4m3_codes, host, normwise, say

pytestmark = pytest.mark.gpu

# a direct-to-LDS tile: K not a multiple of its depth makes both operands packed
TILE = mlk.TileConfig(128, 128, 64, 2, 2, 1, 1, 0, 4, 0)
TILE8 = mlk.TileConfig(128, 128, 128, 2, 2, 1, 1, 0, 4, 0)


@pytest.mark.parametrize("kind", ["bf16", "e4m3"])
def test_noalloc_matches_matmul_two_calls(kind):
    for (M, N, K), seed in (((1000, 776, 1001), 1), ((300, 200, 129), 2)):
        say("noalloc", kind, M, N, K)
        A, B = matmul_inputs(M, N, K, seed=seed, dist="normal")
        C0 = random_c(M, N, seed=seed)
        if kind == "bf16":
            qa, qb = oracle.bf16_encode(A), oracle.bf16_encode(B)
            a, b = from_bf16_codes(qa), from_bf16_codes(qb)
            ref = C0.astype(np.float64) + oracle.matmul_f64(oracle.bf16_decode(qa), oracle.bf16_decode(qb))
            kw, tol, tile = {}, 1e-5, TILE
        else:
            qa, sa = oracle.quantize_e4m3(A)
            qb, sb = oracle.quantize_e4m3(B)
            a, b = from_e4m3_codes(qa), from_e4m3_codes(qb)
            alpha = float(np.float32(sa)) * float(np.float32(sb))
            ref = C0.astype(np.float64) + alpha * oracle.matmul_f64(oracle.e4m3_decode(qa), oracle.e4m3_decode(qb))
            kw = dict(scale_a=dev(np.array([sa], np.float32)), scale_b=dev(np.array([sb], np.float32)))
            tol, tile = 5e-5, TILE8
        assert mlk.config_legal(mlk.matmul_problem(M, N, K, L.MLK_BF16 if kind == "bf16" else L.MLK_F8E4M3,
                                                   L.MLK_F32), tile)
        C1, C2 = dev(C0), dev(C0)
        mlk.matmul(a, b, C1, cfg=tile, **kw)
        mlk.matmul_noalloc(a, b, C2, cfg=tile, **kw)
        g1, g2 = host(C1), host(C2)
        assert np.array_equal(g1, g2), "noalloc differs from mlk_matmul"
        e = normwise(g2, ref)
        say("  normwise vs oracle", e)
        assert e <= tol
        # small integers: exact
        Sa, Sb = matmul_inputs(M, N, K, seed=seed + 10, dist="small_int")
        if kind == "bf16":
            sa_, sb_ = from_bf16_codes(oracle.bf16_encode(Sa)), from_bf16_codes(oracle.bf16_encode(Sb))
        else:
            sa_, sb_ = from_e4m3_codes(oracle.e4m3_encode(Sa, 1.0)), from_e4m3_codes(oracle.e4m3_encode(Sb, 1.0))
        C = torch.zeros(M, N, device="cuda")
        mlk.matmul_noalloc(sa_, sb_, C, cfg=tile)
        assert np.array_equal(host(C).astype(np.float64), oracle.matmul_f64(Sa, Sb))


def test_noalloc_refuses_oversized_packing():
    # A packed as 4096 x 8256 bf16 (66 MiB) plus B: more than the 64 MiB array
    M, N, K = 4096, 64, 8193
    a = torch.zeros(M, K, dtype=torch.bfloat16, device="cuda")
    b = torch.zeros(K, N, dtype=torch.bfloat16, device="cuda")
    C = torch.full((M, N), 3.0, device="cuda")
    with pytest.raises(mlk.MlkError, match="SHAPE"):
        mlk.matmul_noalloc(a, b, C, cfg=TILE)
    assert torch.all(C == 3.0).item()   # nothing was enqueued
    # the same shape without packing work (register-loaded tile) runs
    mlk.matmul_noalloc(a, b, C, cfg=mlk.TileConfig(128, 128, 64, 2, 2, 1, 1, 0, 1, 0))
    assert torch.all(C == 3.0).item()   # zero operands, C += 0
