"""GPU parity of the fp32 chunk-gather conv tiles (stages 1, layout 0: whole K
chunks gathered from NCHW, k decomposed per wave) against the CPU oracle.

Every such tile at split K 1, 2, 4 and 8 (where legal) on ragged shapes:
C = 1, 3 and 7 (K not a multiple of 4: the filter is read element by
element), strides, padding, several images per tile, F and pixel counts that
cut tiles, 1 x 1, 5 x 5 and 7 x 7 filters; C += conv on normal data within
1e-5 normwise of the double result, and overwrite on small integers bit for
bit (every partial sum is exact, whatever the split and order).  Then every
legal configuration of these tiles for the 56 x 56 x 64 3 x 3 layer, exact
on small integers, and the tile picked by exhaustive search against the
oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_16080_amd as mlk
from paper_2307_16080_amd import _lib as L
from workloads import conv_inputs

from gpu_util import dev, host, normwise, say

pytestmark = pytest.mark.gpu

CASES = [
    (1, 3, 17, 19, 5, 3, 3, 1, 1),
    (2, 16, 13, 11, 40, 3, 3, 2, 1),
    (3, 24, 7, 7, 130, 1, 1, 1, 0),
    (2, 32, 20, 20, 64, 5, 5, 2, 2),
    (1, 1, 30, 30, 3, 3, 3, 1, 0),
    (1, 7, 9, 9, 17, 7, 7, 1, 3),
    (2, 64, 14, 14, 65, 3, 3, 1, 1),
]


def _chunk_tiles():
    p = mlk.conv_problem(1, 64, 56, 56, 64, 3, 3, 1, 1, L.MLK_F32, L.MLK_F32)
    seen = {}
    for c in mlk.configs(p):
        if c.stages == 1:
            seen.setdefault((c.bm, c.bn, c.bk, c.wm, c.wn), c)
    return list(seen)


TILES = _chunk_tiles()


def _prob(case):
    N, C, H, W, F, KH, KW, s, p = case
    return mlk.conv_problem(N, C, H, W, F, KH, KW, s, p, L.MLK_F32, L.MLK_F32)


def _yshape(case):
    N, C, H, W, F, KH, KW, s, p = case
    return (N, F, (H + 2 * p - KH) // s + 1, (W + 2 * p - KW) // s + 1)


def test_chunk_tiles_exist():
    assert len(TILES) >= 6, TILES


@pytest.mark.parametrize("tile", TILES, ids=lambda t: "x".join(map(str, t)))
def test_chunk_conv_ragged(tile):
    bm, bn, bk, wm, wn = tile
    for case in CASES:
        N, C, H, W, F, KH, KW, s, p = case
        x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=sum(case))
        xi, wi = conv_inputs(N, C, H, W, F, KH, KW, seed=7, dist="small_int")
        y0 = np.random.default_rng(2).uniform(-1, 1, _yshape(case)).astype(np.float32)
        ref = oracle.conv2d_f64(x, w, (s, s), (p, p), y=y0)
        refi = oracle.conv2d_f64(xi, wi, (s, s), (p, p))
        for split in (1, 2, 4, 8):
            cfg = mlk.TileConfig(bm, bn, bk, wm, wn, split, 1, 0, 1, 0, 0)
            if not mlk.config_legal(_prob(case), cfg):
                continue
            say("chunk conv", tile, "split", split, case)
            y = dev(y0)
            mlk.conv2d_nchw_fchw(dev(x), dev(w), y, (s, s), (p, p), cfg=cfg)
            assert normwise(host(y), ref) <= 1e-5, (case, split)
            yi = torch.full(_yshape(case), float("nan"), device="cuda")
            mlk.conv2d_nchw_fchw(dev(xi), dev(wi), yi, (s, s), (p, p), accumulate=False, cfg=cfg)
            assert np.array_equal(host(yi).astype(np.float64), refi), (case, split)


def test_chunk_conv_56x56x64_every_config():
    case = (1, 64, 56, 56, 64, 3, 3, 1, 1)
    xi, wi = conv_inputs(*case[:7], seed=5, dist="small_int")
    refi = oracle.conv2d_f64(xi, wi, (1, 1), (1, 1), threads=oracle.default_threads())
    xd, wd = dev(xi), dev(wi)
    n = 0
    for cfg in mlk.configs(_prob(case)):
        if cfg.stages != 1:
            continue
        n += 1
        yi = torch.full(_yshape(case), float("nan"), device="cuda")
        mlk.conv2d_nchw_fchw(xd, wd, yi, (1, 1), (1, 1), accumulate=False, cfg=cfg)
        assert np.array_equal(host(yi).astype(np.float64), refi), cfg
        call = mlk.ConvCall(xd, wd, yi, (1, 1), (1, 1), cfg=cfg)
        call()
        assert np.array_equal(host(yi).astype(np.float64), 2.0 * refi), cfg
    say("56x56x64 chunk configurations", n)
    assert n >= 20


def test_chunk_conv_56x56x64_tuned():
    """The exhaustive search's pick for the benchmark's fp32 layer, on its
    normal inputs, within 1e-5 of the double result."""
    case = (1, 64, 56, 56, 64, 3, 3, 1, 1)
    x, w = conv_inputs(*case[:7], seed=0)
    ref = oracle.conv2d_f64(x, w, (1, 1), (1, 1), threads=oracle.default_threads())
    best, _, _ = mlk.tune(_prob(case), mlk.MLK_TUNE_EXHAUSTIVE, reps=3, warmup=1)
    say("tuned fp32 conv", best)
    y = torch.zeros(_yshape(case), device="cuda")
    mlk.conv2d_nchw_fchw(dev(x), dev(w), y, (1, 1), (1, 1), cfg=best)
    assert normwise(host(y), ref) <= 1e-5


def test_chunk_conv_default_for_small_fp32_layers_and_capture():
    """With no configuration the 56 x 56 x 64 fp32 layer (49 tiles of 64 x 64,
    fewer than the CUs) runs the chunk-gather tile, K split 8 ways; the
    per-call route allocates nothing, so it is captured into a graph (the
    split's zero fill is a kernel), and three replays with eager work between
    them each give the oracle's values, bit for bit on small integers."""
    case = (1, 64, 56, 56, 64, 3, 3, 1, 1)
    x, w = conv_inputs(*case[:7], seed=9, dist="small_int")
    ref = oracle.conv2d_f64(x, w, (1, 1), (1, 1), threads=oracle.default_threads())
    xd, wd = dev(x), dev(w)
    y = torch.zeros(_yshape(case), device="cuda")
    # (the overwriting form: the searches elsewhere record their picks as the
    # default of the accumulating one)
    c = mlk.ConvCall(xd, wd, y, (1, 1), (1, 1), accumulate=False).config
    say("default fp32 conv config", c)
    assert (c.bm, c.bn, c.bk, c.stages, c.layout) == (64, 64, 16, 1, 0)
    assert c.split_k == 8
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        mlk.conv2d_nchw_fchw(xd, wd, y, (1, 1), (1, 1), accumulate=False)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert np.array_equal(host(y).astype(np.float64), ref)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mlk.conv2d_nchw_fchw(xd, wd, y, (1, 1), (1, 1), accumulate=False)
    for r in range(3):
        y.fill_(float("nan"))
        junk = torch.randn(1 << 16, device="cuda").sum()
        g.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk).item()
        assert np.array_equal(host(y).astype(np.float64), ref), r
    del g
