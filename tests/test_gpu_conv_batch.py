"""GPU parity of mlk_conv2d_batch_* (many independent convolutions in one
persistent launch of the channel-gather conv tile) against the CPU oracle.

Small-integer operands keep every fp32 partial sum exact whatever the K split
and order, so the batch must equal the oracle bit for bit; normal operands
within 1e-5 normwise of the double result.  Cases: the ResNet-18 conv stack
at batch 1 (19 convolutions, each its own input, as the benchmark's stack),
ragged shapes (strides, padding, F and pixel counts that cut tiles, 1 x 1 and
5 x 5 filters), overwrite and accumulate, every persistent tile with split
caps 1 and 16, replays of a captured graph of the batch, a filter update, and
the batch-32 stack in the benchmark's configuration on sampled images.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_16080_amd as mlk
from workloads import conv_inputs, resnet18_conv_stack

from gpu_util import dev, from_bf16_codes, host, normwise, say

pytestmark = pytest.mark.gpu

RAGGED = [
    (1, 8, 9, 9, 5, 3, 3, 1, 1),
    (3, 16, 13, 11, 40, 3, 3, 2, 1),
    (2, 64, 14, 14, 65, 3, 3, 1, 1),
    (5, 24, 7, 7, 130, 1, 1, 1, 0),
    (2, 32, 20, 20, 64, 5, 5, 2, 2),
    (1, 128, 16, 16, 64, 1, 1, 2, 0),
]


def _resnet_b1():
    out = []
    for shape, count in resnet18_conv_stack(1):
        out += [(shape.N, shape.C, shape.H, shape.W, shape.F, shape.KH, shape.KW, shape.stride, shape.pad)] * count
    return out


def _tiles():
    return [mlk.TileConfig(c.bm, c.bn, 64, c.wm, c.wn, 16, 1, 0, 1, 3)
            for c in {(c.bm, c.bn, c.wm, c.wn): c for c in mlk.configs(mlk.conv_problem(1, 64, 56, 56, 64, 3, 3, 1, 1))
                      if c.layout == 3}.values()]


def _make(cases, dist, seed):
    """Device operands and exact-or-double references for each case."""
    ops = []
    for i, (N, C, H, W, F, KH, KW, s, p) in enumerate(cases):
        x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=seed + i, dist=dist)
        qx, qw = oracle.bf16_encode(x), oracle.bf16_encode(w)
        ho, wo = (H + 2 * p - KH) // s + 1, (W + 2 * p - KW) // s + 1
        y0 = np.random.default_rng(seed + 1000 + i).uniform(-1, 1, (N, F, ho, wo)).astype(np.float32)
        if dist == "small_int":
            y0 = np.rint(y0 * 8)
        ops.append(dict(x=from_bf16_codes(qx), w=from_bf16_codes(qw), xv=oracle.bf16_decode(qx),
                        wv=oracle.bf16_decode(qw), y0=y0, stride=(s, s), pad=(p, p)))
    return ops


def _run_and_check(ops, accumulate, cfg, exact, threads=8):
    ys = [dev(o["y0"]) if accumulate else torch.full(o["y0"].shape, float("nan"), device="cuda") for o in ops]
    batch = mlk.ConvBatch([(o["x"], o["w"], y, o["stride"], o["pad"]) for o, y in zip(ops, ys)],
                          accumulate=accumulate, cfg=cfg)
    c, tasks, wgs = batch.info()
    say("  batch", c, "tasks", tasks, "workgroups", wgs)
    batch()
    for i, (o, y) in enumerate(zip(ops, ys)):
        ref = oracle.conv2d_f64(o["xv"], o["wv"], o["stride"], o["pad"], y=o["y0"] if accumulate else None,
                                threads=threads)
        got = host(y).astype(np.float64)
        if exact:
            assert np.array_equal(got, ref), (i, accumulate)
        else:
            assert normwise(got, ref) <= 1e-5, (i, accumulate, normwise(got, ref))
    return batch, ys


@pytest.mark.parametrize("cfg", _tiles(), ids=lambda c: f"{c.bm}x{c.bn}_{c.wm}{c.wn}")
def test_conv_batch_ragged_every_tile(cfg):
    for cap in (1, 16):
        c = mlk.TileConfig(cfg.bm, cfg.bn, 64, cfg.wm, cfg.wn, cap, 1, 0, 1, 3)
        say("conv batch ragged", c)
        ops = _make(RAGGED, "small_int", seed=11)
        for acc in (True, False):
            _run_and_check(ops, acc, c, exact=True)
    _run_and_check(_make(RAGGED, "normal", seed=12), True, cfg, exact=False)


def test_conv_batch_resnet18_b1_default():
    cases = _resnet_b1()
    assert len(cases) == 19
    say("conv batch resnet18 b1, small integers")
    for acc in (True, False):
        _run_and_check(_make(cases, "small_int", seed=21), acc, None, exact=True)
    say("conv batch resnet18 b1, normal")
    _run_and_check(_make(cases, "normal", seed=22), True, None, exact=False)


def test_conv_batch_resnet18_b1_benchmark_grid():
    """Every configuration the benchmark times the b1 batch in (64 x 64, 64 x 128
    and 128 x 128 tiles, split caps 1, 4, 16, 32), exact on small integers."""
    ops = _make(_resnet_b1(), "small_int", seed=23)
    refs = [oracle.conv2d_f64(o["xv"], o["wv"], o["stride"], o["pad"], threads=8) for o in ops]
    for bm, bn in ((64, 64), (64, 128), (128, 128)):
        for cap in (1, 4, 16, 32):
            cfg = mlk.TileConfig(bm, bn, 64, 2, 2, cap, 1, 0, 1, 3)
            ys = [torch.full(o["y0"].shape, float("nan"), device="cuda") for o in ops]
            batch = mlk.ConvBatch([(o["x"], o["w"], y, o["stride"], o["pad"]) for o, y in zip(ops, ys)],
                                  accumulate=False, cfg=cfg)
            batch()
            for i, (y, ref) in enumerate(zip(ys, refs)):
                assert np.array_equal(host(y).astype(np.float64), ref), (cfg, i)


def test_conv_batch_graph_replays_and_filter_update():
    """The batch captured into a graph (zero fills and persistent launch),
    replayed three times with eager work between replays: each replay equals
    the eager result; then the filters change in place and update_filters
    makes the next replay use them."""
    cases = RAGGED + _resnet_b1()[-4:]
    ops = _make(cases, "small_int", seed=31)
    ys = [torch.full(o["y0"].shape, float("nan"), device="cuda") for o in ops]
    batch = mlk.ConvBatch([(o["x"], o["w"], y, o["stride"], o["pad"]) for o, y in zip(ops, ys)],
                          accumulate=False)
    refs = [oracle.conv2d_f64(o["xv"], o["wv"], o["stride"], o["pad"], threads=8) for o in ops]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batch()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch()
    for r in range(3):
        for y in ys:
            y.fill_(float("nan"))
        scratch = torch.randn(1 << 20, device="cuda").sum()     # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(scratch).item()
        for i, (y, ref) in enumerate(zip(ys, refs)):
            assert np.array_equal(host(y).astype(np.float64), ref), (r, i)
    # new filter values in place: stale until update_filters
    for o in ops:
        o["w"].copy_(-o["w"])
    batch.update_filters()
    g.replay()
    torch.cuda.synchronize()
    for i, (y, ref) in enumerate(zip(ys, refs)):
        assert np.array_equal(host(y).astype(np.float64), -ref), i


def test_conv_batch_resnet18_b32_sampled_images():
    """The b32 stack's 19 convolutions as one batch, in the configuration the
    benchmark times at batch 32 (64 x 64 tile, no split) and the default one:
    images 0 and 31 of every output against the oracle on those images alone
    (a convolution treats each image on its own), small integers exact, and
    every output finite."""
    cases = []
    for shape, count in resnet18_conv_stack(32):
        cases += [(shape.N, shape.C, shape.H, shape.W, shape.F, shape.KH, shape.KW, shape.stride, shape.pad)] * count
    ops = []
    for i, (N, C, H, W, F, KH, KW, s, p) in enumerate(cases):
        rng = np.random.default_rng(40 + i)
        x = rng.integers(-4, 5, (N, C, H, W)).astype(np.float32)
        w = rng.integers(-4, 5, (F, C, KH, KW)).astype(np.float32)
        ho, wo = (H + 2 * p - KH) // s + 1, (W + 2 * p - KW) // s + 1
        ops.append(dict(x=from_bf16_codes(oracle.bf16_encode(x)), w=from_bf16_codes(oracle.bf16_encode(w)),
                        xs=x[[0, N - 1]], wv=w, shape=(N, F, ho, wo), stride=(s, s), pad=(p, p)))
    refs = [oracle.conv2d_f64(o["xs"], o["wv"], o["stride"], o["pad"], threads=8) for o in ops]
    for cfg in (mlk.TileConfig(64, 64, 64, 2, 2, 1, 1, 0, 1, 3), None):
        say("conv batch resnet18 b32", cfg)
        ys = [torch.full(o["shape"], float("nan"), device="cuda") for o in ops]
        batch = mlk.ConvBatch([(o["x"], o["w"], y, o["stride"], o["pad"]) for o, y in zip(ops, ys)],
                              accumulate=False, cfg=cfg)
        batch()
        for i, (y, ref) in enumerate(zip(ys, refs)):
            assert torch.isfinite(y).all().item(), i
            got = host(y[[0, y.shape[0] - 1]]).astype(np.float64)
            assert np.array_equal(got, ref), (i, cfg)
