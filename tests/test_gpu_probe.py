"""GPU check of the MFMA rate probe (mlk_mfma_rate): every wave's result is
exact (all-ones operands: 28 + 8 * iters * k, k = 32 for bf16, 128 for
e4m3), the flop count is the launch's, and the rate is below the datasheet
peak."""
import pytest
import torch

import paper_2307_16080_amd as mlk

from gpu_util import say

pytestmark = pytest.mark.gpu

PEAK = {"bf16": 2516.6e12, "e4m3": 5033.2e12}


@pytest.mark.parametrize("dtype,k", [("bf16", 32), ("e4m3", 128)])
def test_mfma_rate_exact_and_below_peak(dtype, k):
    cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    for iters in (1, 7, 256):
        flops, out = mlk.mfma_rate(dtype, iters)
        torch.cuda.synchronize()
        assert out.numel() == 8 * cus
        assert flops == 8 * cus * iters * 8 * 2 * 16 * 16 * k
        assert torch.all(out == float(28 + 8 * iters * k)).item(), (dtype, iters, out[:4].tolist())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    mlk.mfma_rate(dtype, 1024)
    e0.record()
    for _ in range(5):
        flops, _ = mlk.mfma_rate(dtype, 1024)
    e1.record()
    torch.cuda.synchronize()
    rate = 5 * flops / (e0.elapsed_time(e1) * 1e-3)
    say(dtype, "MFMA rate", rate / 1e12, "TFLOP/s")
    assert 0 < rate <= 1.02 * PEAK[dtype]
