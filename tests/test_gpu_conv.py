"""GPU parity of the implicit-GEMM conv2d (fp32 and bf16 inputs) against the
oracle's direct NCHW x FCHW loop nest: normwise <= 1e-5 against the double
result on the same (quantised) inputs, bit-exact on small-integer inputs.
Covers the fp32 56x56x64 workload, stride 2, padding, 1x1 filters, batch > 1,
odd sizes, every compiled conv tile, and the ResNet-18 layer shapes in bf16.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2307_16080_amd as mlk
from paper_2307_16080_amd import _lib as L
from workloads import CFG_CONV_F32, conv_inputs, matmul_inputs, resnet18_conv_stack

from gpu_util import all_tiles, dev, from_bf16_codes, host, normwise, say

pytestmark = pytest.mark.gpu

CASES = [
    # N, C, H, W, F, KH, KW, stride, pad
    (1, 3, 7, 6, 2, 3, 3, 1, 1),
    (2, 5, 9, 11, 7, 3, 3, 2, 1),
    (1, 16, 8, 8, 33, 1, 1, 2, 0),
    (3, 4, 13, 13, 20, 5, 5, 1, 2),
    (1, 1, 40, 40, 3, 3, 3, 1, 0),
    (2, 64, 14, 14, 65, 3, 3, 1, 1),
]


def _out(x, w, s, p):
    N, C, H, W = x.shape
    F, _, KH, KW = w.shape
    return torch.zeros(N, F, (H + 2 * p - KH) // s + 1, (W + 2 * p - KW) // s + 1, device="cuda")


def test_f32_conv_56x56x64():
    sh = CFG_CONV_F32
    x, w = conv_inputs(sh.N, sh.C, sh.H, sh.W, sh.F, sh.KH, sh.KW, seed=0)
    ref = oracle.conv2d_f64(x, w, (1, 1), (1, 1), threads=oracle.default_threads())
    y = _out(x, w, 1, 1)
    mlk.conv2d_nchw_fchw(dev(x), dev(w), y, (1, 1), (1, 1))
    err = normwise(host(y), ref)
    say("f32 conv 56x56x64 normwise", err)
    assert err <= 1e-5


@pytest.mark.parametrize("cfg", all_tiles(L.MLK_F32, L.MLK_F32, conv=True) + all_tiles(L.MLK_BF16, L.MLK_F32, conv=True),
                         ids=lambda c: f"{c.bm}x{c.bn}x{c.bk}_{c.wm}{c.wn}_l{c.layout}")
def test_every_conv_tile(cfg):
    for case in CASES:
        N, C, H, W, F, KH, KW, s, p = case
        say("conv", cfg, case)
        for is_bf16 in (False, True):
            try_cfg = cfg
            if not mlk.config_legal(mlk.conv_problem(N, C, H, W, F, KH, KW, s, p,
                                                     L.MLK_BF16 if is_bf16 else L.MLK_F32, L.MLK_F32), try_cfg):
                continue
            x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=sum(case))
            y0 = np.random.default_rng(1).uniform(-1, 1, (N, F, (H + 2 * p - KH) // s + 1,
                                                          (W + 2 * p - KW) // s + 1)).astype(np.float32)
            if is_bf16:
                qx, qw = oracle.bf16_encode(x), oracle.bf16_encode(w)
                ref = oracle.conv2d_f64(oracle.bf16_decode(qx), oracle.bf16_decode(qw), (s, s), (p, p), y=y0)
                xd, wd = from_bf16_codes(qx), from_bf16_codes(qw)
            else:
                ref = oracle.conv2d_f64(x, w, (s, s), (p, p), y=y0)
                xd, wd = dev(x), dev(w)
            y = dev(y0)
            mlk.conv2d_nchw_fchw(xd, wd, y, (s, s), (p, p), cfg=try_cfg)
            assert normwise(host(y), ref) <= 1e-5, (case, is_bf16)
            # small integers: exact
            x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=3, dist="small_int")
            y = _out(x, w, s, p)
            if is_bf16:
                mlk.conv2d_nchw_fchw(from_bf16_codes(oracle.bf16_encode(x)),
                                     from_bf16_codes(oracle.bf16_encode(w)), y, (s, s), (p, p),
                                     cfg=try_cfg)
            else:
                mlk.conv2d_nchw_fchw(dev(x), dev(w), y, (s, s), (p, p), cfg=try_cfg)
            assert np.array_equal(host(y).astype(np.float64), oracle.conv2d_f64(x, w, (s, s), (p, p))), case


FAST_CONV = [c for c in all_tiles(L.MLK_BF16, L.MLK_F32, conv=True) if c.stages == 1 and c.layout == 1]
GATHER_CONV = [c for c in all_tiles(L.MLK_BF16, L.MLK_F32, conv=True) if c.layout == 3]
# channels-last shapes (C a multiple of 8): strides, padding, K = C*KH*KW not a
# multiple of the 64-deep stage, tiles that span images, ragged F and pixels
FAST_CASES = [
    (1, 8, 9, 9, 5, 3, 3, 1, 1),
    (3, 16, 13, 11, 40, 3, 3, 2, 1),
    (2, 64, 14, 14, 65, 3, 3, 1, 1),
    (5, 24, 7, 7, 130, 1, 1, 1, 0),
    (2, 32, 20, 20, 64, 5, 5, 2, 2),
    # H*W and C multiples of 8 (the 16-byte transpose), ragged against its 64 x 64 tiles
    (2, 72, 10, 20, 24, 3, 3, 1, 1),
    (1, 128, 16, 16, 64, 1, 1, 1, 0),
]


@pytest.mark.parametrize("cfg", FAST_CONV, ids=lambda c: f"{c.bm}x{c.bn}x{c.bk}_{c.wm}{c.wn}")
def test_fast_conv_tiles(cfg):
    assert cfg.layout == 1
    with pytest.raises(mlk.MlkError, match="CONFIG"):    # no NCHW form of this tile
        x = torch.zeros(1, 8, 4, 4, dtype=torch.bfloat16, device="cuda")
        mlk.conv2d_nchw_fchw(x, torch.zeros(8, 8, 3, 3, dtype=torch.bfloat16, device="cuda"),
                             torch.zeros(1, 8, 2, 2, device="cuda"), (1, 1), (0, 0),
                             cfg=mlk.TileConfig(*list(cfg.as_tuple())[:9], 0))
    for case in FAST_CASES:
        N, C, H, W, F, KH, KW, s, p = case
        say("fast conv", cfg, case)
        x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=sum(case) + 1)
        ho, wo = (H + 2 * p - KH) // s + 1, (W + 2 * p - KW) // s + 1
        y0 = np.random.default_rng(2).uniform(-1, 1, (N, F, ho, wo)).astype(np.float32)
        qx, qw = oracle.bf16_encode(x), oracle.bf16_encode(w)
        ref = oracle.conv2d_f64(oracle.bf16_decode(qx), oracle.bf16_decode(qw), (s, s), (p, p), y=y0)
        y = dev(y0)
        mlk.conv2d_nchw_fchw(from_bf16_codes(qx), from_bf16_codes(qw), y, (s, s), (p, p), cfg=cfg)
        assert normwise(host(y), ref) <= 1e-5, case
        x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=4, dist="small_int")
        for acc in (True, False):
            y = torch.full((N, F, ho, wo), float("nan"), device="cuda") if not acc else \
                torch.zeros(N, F, ho, wo, device="cuda")
            mlk.conv2d_nchw_fchw(from_bf16_codes(oracle.bf16_encode(x)), from_bf16_codes(oracle.bf16_encode(w)),
                                 y, (s, s), (p, p), cfg=cfg, accumulate=acc)
            assert np.array_equal(host(y).astype(np.float64), oracle.conv2d_f64(x, w, (s, s), (p, p))), (case, acc)


@pytest.mark.parametrize("cfg", GATHER_CONV, ids=lambda c: f"{c.bm}x{c.bn}x{c.bk}_{c.wm}{c.wn}")
def test_gather_conv_tiles(cfg):
    """Layout 3: the register-loaded conv tile reading the NCHW input itself
    (8 channels of a pixel gathered per 16-byte chunk), per call (the filter
    transposed in scratch memory, or used as it is when 1 x 1) and bound
    (mlk.ConvCall: the filter transposed once), overwrite and accumulate, with
    split K; C not a multiple of 8 is refused."""
    assert GATHER_CONV and cfg.stages == 1
    assert not mlk.config_legal(mlk.conv_problem(1, 12, 8, 8, 16, 3, 3, 1, 1, L.MLK_BF16, L.MLK_F32), cfg)
    for case in FAST_CASES:
        N, C, H, W, F, KH, KW, s, p = case
        say("gather conv", cfg, case)
        prob = mlk.conv_problem(N, C, H, W, F, KH, KW, s, p, L.MLK_BF16, L.MLK_F32)
        x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=sum(case) + 11)
        ho, wo = (H + 2 * p - KH) // s + 1, (W + 2 * p - KW) // s + 1
        y0 = np.random.default_rng(5).uniform(-1, 1, (N, F, ho, wo)).astype(np.float32)
        qx, qw = oracle.bf16_encode(x), oracle.bf16_encode(w)
        ref = oracle.conv2d_f64(oracle.bf16_decode(qx), oracle.bf16_decode(qw), (s, s), (p, p), y=y0)
        y = dev(y0)
        mlk.conv2d_nchw_fchw(from_bf16_codes(qx), from_bf16_codes(qw), y, (s, s), (p, p), cfg=cfg)
        assert normwise(host(y), ref) <= 1e-5, case
        xi, wi = conv_inputs(N, C, H, W, F, KH, KW, seed=6, dist="small_int")
        exact = oracle.conv2d_f64(xi, wi, (s, s), (p, p))
        dx, dw = from_bf16_codes(oracle.bf16_encode(xi)), from_bf16_codes(oracle.bf16_encode(wi))
        for sk in (1, 2):
            c = mlk.TileConfig(cfg.bm, cfg.bn, cfg.bk, cfg.wm, cfg.wn, sk, 1, 0, 1, 3)
            if not mlk.config_legal(prob, c):
                continue
            for acc in (True, False):
                y = torch.zeros(N, F, ho, wo, device="cuda") if acc else \
                    torch.full((N, F, ho, wo), float("nan"), device="cuda")
                mlk.conv2d_nchw_fchw(dx, dw, y, (s, s), (p, p), cfg=c, accumulate=acc)
                assert np.array_equal(host(y).astype(np.float64), exact), (case, sk, acc)
            # bound: one launch per call, the filter transposed at creation
            y = torch.full((N, F, ho, wo), float("nan"), device="cuda")
            call = mlk.ConvCall(dx, dw, y, (s, s), (p, p), cfg=c, accumulate=False)
            assert call.config.layout == 3
            call()
            call()
            assert np.array_equal(host(y).astype(np.float64), exact), (case, sk, "plan")


FAST_CONV_DMA = [c for c in all_tiles(L.MLK_BF16, L.MLK_F32, conv=True) if c.stages >= 2]
# channels-last shapes with C*KH*KW a multiple of the 64-deep stage: C below,
# equal to and above the stage (several taps per stage, one tap, one tap over
# several stages), strides, padding, ragged F and pixels, tiles across images
DMA_CASES = [
    (1, 8, 16, 16, 5, 4, 2, 1, 0),
    (2, 16, 9, 9, 33, 2, 2, 1, 1),
    (2, 64, 14, 14, 65, 3, 3, 1, 1),
    (3, 64, 13, 11, 40, 3, 3, 2, 1),
    (1, 128, 16, 16, 64, 1, 1, 1, 0),
    (4, 128, 7, 7, 130, 3, 3, 1, 1),
]


@pytest.mark.parametrize("cfg", FAST_CONV_DMA, ids=lambda c: f"{c.bm}x{c.bn}x{c.bk}_{c.wm}{c.wn}_s{c.stages}")
def test_fast_conv_dma_tiles(cfg):
    assert cfg.layout == 1 and FAST_CONV_DMA
    # depth not a multiple of the stage: refused
    assert not mlk.config_legal(mlk.conv_problem(1, 24, 8, 8, 16, 3, 3, 1, 1, L.MLK_BF16, L.MLK_F32), cfg)
    for case in DMA_CASES:
        N, C, H, W, F, KH, KW, s, p = case
        say("dma conv", cfg, case)
        x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=sum(case) + 7)
        ho, wo = (H + 2 * p - KH) // s + 1, (W + 2 * p - KW) // s + 1
        y0 = np.random.default_rng(3).uniform(-1, 1, (N, F, ho, wo)).astype(np.float32)
        qx, qw = oracle.bf16_encode(x), oracle.bf16_encode(w)
        ref = oracle.conv2d_f64(oracle.bf16_decode(qx), oracle.bf16_decode(qw), (s, s), (p, p), y=y0)
        y = dev(y0)
        mlk.conv2d_nchw_fchw(from_bf16_codes(qx), from_bf16_codes(qw), y, (s, s), (p, p), cfg=cfg)
        assert normwise(host(y), ref) <= 1e-5, case
        x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=5, dist="small_int")
        for acc in (True, False):
            y = torch.full((N, F, ho, wo), float("nan"), device="cuda") if not acc else \
                torch.zeros(N, F, ho, wo, device="cuda")
            mlk.conv2d_nchw_fchw(from_bf16_codes(oracle.bf16_encode(x)), from_bf16_codes(oracle.bf16_encode(w)),
                                 y, (s, s), (p, p), cfg=cfg, accumulate=acc)
            assert np.array_equal(host(y).astype(np.float64), oracle.conv2d_f64(x, w, (s, s), (p, p))), (case, acc)


def test_conv_split_k_overwrite():
    x, w = conv_inputs(1, 64, 14, 14, 32, 3, 3, seed=4, dist="small_int")
    ref = oracle.conv2d_f64(x, w, (1, 1), (1, 1))
    for layout in (0, 1):
        for sk in (1, 2, 4):
            y = torch.full((1, 32, 14, 14), float("nan"), device="cuda")
            mlk.conv2d_nchw_fchw(dev(x), dev(w), y, (1, 1), (1, 1), accumulate=False,
                                 cfg=mlk.TileConfig(32, 32, 16, 1, 1, sk, 1, 0, 0, layout))
            assert np.array_equal(host(y).astype(np.float64), ref), (layout, sk)


@pytest.mark.parametrize("batch", [1, 2])
def test_resnet18_layers_bf16(batch):
    for shape, _count in resnet18_conv_stack(batch):
        say("resnet layer", shape)
        x, w = conv_inputs(shape.N, shape.C, shape.H, shape.W, shape.F, shape.KH, shape.KW, seed=shape.C)
        qx, qw = oracle.bf16_encode(x), oracle.bf16_encode(w)
        ref = oracle.conv2d_f64(oracle.bf16_decode(qx), oracle.bf16_decode(qw), (shape.stride,) * 2,
                                (shape.pad,) * 2, threads=oracle.default_threads())
        y = torch.zeros(ref.shape, device="cuda")
        mlk.conv2d_nchw_fchw(from_bf16_codes(qx), from_bf16_codes(qw), y, (shape.stride,) * 2,
                             (shape.pad,) * 2)
        assert normwise(host(y), ref) <= 1e-5


def test_paper_conv_shape_f32():
    """The paper's measured workload: one 1280x1280 image, 3 output channels, 3x3, valid."""
    x, w = conv_inputs(1, 1, 1280, 1280, 3, 3, 3, seed=0)
    ref = oracle.conv2d_f64(x, w, threads=oracle.default_threads())
    y = torch.zeros(1, 3, 1278, 1278, device="cuda")
    mlk.conv2d_nchw_fchw(dev(x), dev(w), y)
    assert normwise(host(y), ref) <= 1e-5


def test_workspace_routes_refused_under_capture():
    """On a capturing stream the routes that take a stream-ordered workspace
    (channels-last conv, packed direct-to-LDS matmul) return MLK_ERR_CONFIG
    and record nothing; the capture itself stays valid."""
    x = torch.zeros(1, 64, 8, 8, dtype=torch.bfloat16, device="cuda")
    w = torch.zeros(64, 64, 3, 3, dtype=torch.bfloat16, device="cuda")
    y = torch.zeros(1, 64, 8, 8, device="cuda")
    A = torch.zeros(40, 72, dtype=torch.bfloat16, device="cuda")
    B = torch.zeros(72, 24, dtype=torch.bfloat16, device="cuda")
    C = torch.zeros(40, 24, device="cuda")
    t = torch.zeros(16, device="cuda")
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        t.add_(1.0)
        with pytest.raises(mlk.MlkError, match="CONFIG"):
            mlk.conv2d_nchw_fchw(x, w, y, (1, 1), (1, 1), cfg=mlk.TileConfig(128, 128, 64, 2, 2, 1, 1, 0, 1, 1))
        with pytest.raises(mlk.MlkError, match="CONFIG"):
            mlk.matmul(A, B, C, cfg=mlk.TileConfig(128, 128, 64, 2, 2, 1, 1, 0, 2, 0))
        # the channel gather transposes a 3 x 3 filter into scratch memory
        with pytest.raises(mlk.MlkError, match="CONFIG"):
            mlk.conv2d_nchw_fchw(x, w, y, (1, 1), (1, 1), cfg=mlk.TileConfig(64, 64, 64, 2, 2, 1, 1, 0, 1, 3))
        # a defaulted conv whose default is the channel gather takes the plain tile instead
        mlk.conv2d_nchw_fchw(x, w, y, (1, 1), (1, 1))
    del graph
    torch.cuda.synchronize()


def test_conv_stack_graph_capture_replays():
    """Bound convolutions (mlk.ConvCall: plans whose buffers are allocated when
    they are created) recorded into one HIP graph with torch's capture of the
    current stream: channels-last layers (3 x 3 and 1 x 1, their NHWC copies
    in the plans' own buffers, filters transposed once), an NCHW layer, a
    direct-conv layer, and a packed direct-to-LDS matmul through
    mlk_matmul_noalloc; each layer twice (y += twice).  Every replay, from
    zeroed outputs and with eager work and synchronisations between replays,
    equals the eager calls bit for bit, and the first layer matches the
    oracle."""
    layers = [((2, 64, 14, 14, 64, 3, 3, 1, 1), mlk.TileConfig(128, 128, 64, 2, 2, 1, 1, 0, 1, 1)),
              ((2, 32, 9, 11, 16, 3, 3, 2, 1), mlk.TileConfig(64, 64, 32, 2, 2, 1, 1, 0, 0, 0)),
              ((1, 128, 7, 7, 256, 1, 1, 1, 0), mlk.TileConfig(64, 128, 64, 2, 2, 1, 1, 0, 1, 1)),
              ((1, 64, 56, 56, 64, 3, 3, 1, 1), mlk.TileConfig(64, 64, 64, 2, 2, 1, 1, 0, 3, 1)),
              ((1, 8, 40, 40, 3, 3, 3, 1, 0), None)]
    ops, outs, first = [], [], None
    for i, (case, cfg) in enumerate(layers):
        N, C, H, W, F, KH, KW, s, p = case
        x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=30 + i)
        qx, qw = from_bf16_codes(oracle.bf16_encode(x)), from_bf16_codes(oracle.bf16_encode(w))
        if i == 4:   # fp32 few-filter layer: the direct conv
            qx, qw = dev(x), dev(w)
        y = torch.zeros(N, F, (H + 2 * p - KH) // s + 1, (W + 2 * p - KW) // s + 1, device="cuda")
        call = mlk.ConvCall(qx, qw, y, (s, s), (p, p), cfg=cfg)
        if i == 0:
            first = (x, w, s, p, y)
        ops += [call, call]
        outs.append(y)
    A, B = (from_bf16_codes(oracle.bf16_encode(m)) for m in matmul_inputs(200, 136, 72, seed=5))
    Cm = torch.zeros(200, 136, device="cuda")
    ops.append(lambda: mlk.matmul_noalloc(A, B, Cm, cfg=mlk.TileConfig(128, 128, 64, 2, 2, 1, 1, 0, 4, 0)))
    outs.append(Cm)

    def zero():
        for t in outs:
            t.zero_()

    zero()
    for op in ops:
        op()
    torch.cuda.synchronize()
    want = [t.cpu().clone() for t in outs]
    x, w, s, p, _ = first
    ref = 2.0 * oracle.conv2d_f64(oracle.bf16_decode(oracle.bf16_encode(x)),
                                  oracle.bf16_decode(oracle.bf16_encode(w)), (s, s), (p, p))
    assert normwise(want[0].numpy(), ref) <= 1e-5
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                           # warm-up on a side stream
        for op in ops:
            op()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for op in ops:
            op()
    for rep in range(3):
        zero()
        junk = torch.randn(4096, device="cuda").sum()        # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for i, (t, r) in enumerate(zip(outs, want)):
            assert torch.equal(t.cpu(), r), (rep, i)
        del junk
    del graph


@pytest.mark.parametrize("case", [(2, 64, 14, 14, 64, 3, 3, 1, 1), (1, 128, 7, 7, 256, 1, 1, 2, 0),
                                  (3, 16, 9, 13, 24, 3, 3, 2, 1)])
def test_conv_plan_every_config(case):
    """Every legal configuration of a layer, bound as a plan, equals the per-call
    API bit for bit over two accumulating runs and matches the oracle; the
    filter's values are the ones at binding until update_filter()."""
    N, C, H, W, F, KH, KW, s, p = case
    x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=N + C + F)
    qx, qw = from_bf16_codes(oracle.bf16_encode(x)), from_bf16_codes(oracle.bf16_encode(w))
    ref = oracle.conv2d_f64(oracle.bf16_decode(oracle.bf16_encode(x)), oracle.bf16_decode(oracle.bf16_encode(w)),
                            (s, s), (p, p))
    ho, wo = (H + 2 * p - KH) // s + 1, (W + 2 * p - KW) // s + 1
    prob = mlk.conv_problem(N, C, H, W, F, KH, KW, s, p, L.MLK_BF16, L.MLK_F32)
    for cfg in mlk.configs(prob):
        y1 = torch.zeros(N, F, ho, wo, device="cuda")
        y2 = torch.zeros_like(y1)
        call = mlk.ConvCall(qx, qw, y1, (s, s), (p, p), cfg=cfg)
        assert call.config.as_tuple() == cfg.as_tuple()
        for _ in range(2):
            call()
            mlk.conv2d_nchw_fchw(qx, qw, y2, (s, s), (p, p), cfg=cfg)
        torch.cuda.synchronize()
        if cfg.split_k == 1:   # (split K adds partials with atomics: equal within rounding only)
            assert torch.equal(y1, y2), cfg
        assert normwise(host(y1), 2.0 * ref) <= 1e-5, cfg
        assert normwise(host(y2), 2.0 * ref) <= 1e-5, cfg
    # the bound filter: changed values reach the plan only through update_filter
    # (one configuration of each layout: the channels-last and channel-gather
    # plans hold a transposed copy of a filter larger than 1 x 1)
    firsts = {}
    for c in mlk.configs(prob):
        firsts.setdefault(c.layout, c)
    for cfg in firsts.values():
        call = mlk.ConvCall(qx, qw, y1, (s, s), (p, p), cfg=cfg)
        w_saved = qw.clone()
        qw.zero_()
        y1.zero_()
        call.update_filter()
        call()
        assert torch.count_nonzero(y1).item() == 0, cfg
        qw.copy_(w_saved)
        call.update_filter()
        y1.zero_()
        call()
        assert normwise(host(y1), ref) <= 1e-5, cfg



def test_scratch_shared_across_streams():
    """The workspace routes share one library scratch buffer per device: calls
    interleaved on two streams (growing the buffer on the way) give the same
    bits as the same calls made one after another on the default stream."""
    convs = []
    for i, case in enumerate([(1, 64, 12, 12, 32, 3, 3, 1, 1), (4, 128, 20, 20, 64, 3, 3, 1, 1),
                              (2, 64, 30, 30, 64, 1, 1, 2, 0)]):
        N, C, H, W, F, KH, KW, s, p = case
        x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=40 + i)
        qx, qw = from_bf16_codes(oracle.bf16_encode(x)), from_bf16_codes(oracle.bf16_encode(w))
        convs.append((qx, qw, (s, s), (p, p), (N, F, (H + 2 * p - KH) // s + 1, (W + 2 * p - KW) // s + 1)))
    mms = []
    for i, (M, N, K) in enumerate([(96, 40, 70), (300, 136, 200), (64, 24, 33)]):
        A, B = (from_bf16_codes(oracle.bf16_encode(m)) for m in matmul_inputs(M, N, K, seed=50 + i))
        mms.append((A, B, (M, N)))
    ccfg = mlk.TileConfig(128, 128, 64, 2, 2, 1, 1, 0, 1, 1)
    mcfg = mlk.TileConfig(128, 128, 64, 2, 2, 1, 1, 0, 2, 0)

    def run_all(stream_of):
        outs = []
        for k in range(6):
            x, w, s, p, shp = convs[k % 3]
            A, B, mn = mms[k % 3]
            with torch.cuda.stream(stream_of(k)):
                y = torch.zeros(shp, device="cuda")
                mlk.conv2d_nchw_fchw(x, w, y, s, p, cfg=ccfg)
                C = torch.zeros(mn, device="cuda")
                mlk.matmul(A, B, C, cfg=mcfg)
                outs += [y, C]
        torch.cuda.synchronize()
        return [t.cpu() for t in outs]

    mlk.release()                                            # start from no scratch buffer
    want = run_all(lambda k: torch.cuda.current_stream())
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    mlk.release()
    got = run_all(lambda k: s1 if k % 2 == 0 else s2)
    for i, (a, b) in enumerate(zip(want, got)):
        assert torch.equal(a, b), i


DIRECT_CASES = [
    # N, C, H, W, F, KH, KW, stride, pad: few filters, odd sizes, strides 1-2, taps up to 7x7,
    # images narrower and wider than one 64-pixel row segment, several channels and images
    (1, 1, 37, 70, 3, 3, 3, 1, 0),
    (2, 3, 33, 129, 16, 3, 3, 2, 1),
    (1, 5, 20, 20, 1, 5, 5, 1, 2),
    (3, 2, 11, 9, 7, 7, 7, 1, 3),
    (1, 4, 66, 65, 8, 1, 1, 2, 0),
    (2, 16, 17, 30, 12, 3, 1, 1, 1),
]


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_direct_conv_tiles(dt):
    """The direct (stencil) conv, every compiled tile height, against the
    oracle: normwise <= 1e-5 from a random y (C += conv), bit-exact on small
    integers, and with y overwritten (NaN-filled before)."""
    in_dt = L.MLK_F32 if dt == "f32" else L.MLK_BF16
    for case in DIRECT_CASES:
        N, C, H, W, F, KH, KW, s, p = case
        tiles = [c for c in mlk.configs(mlk.conv_problem(N, C, H, W, F, KH, KW, s, p, in_dt, L.MLK_F32))
                 if c.layout == 2]
        assert sorted(c.bm for c in tiles) == [4, 8, 16, 32], case   # every tile height
        x, w = conv_inputs(N, C, H, W, F, KH, KW, seed=sum(case))
        ho, wo = (H + 2 * p - KH) // s + 1, (W + 2 * p - KW) // s + 1
        y0 = np.random.default_rng(5).uniform(-1, 1, (N, F, ho, wo)).astype(np.float32)
        if dt == "bf16":
            qx, qw = oracle.bf16_encode(x), oracle.bf16_encode(w)
            xv, wv = oracle.bf16_decode(qx), oracle.bf16_decode(qw)
            xd, wd = from_bf16_codes(qx), from_bf16_codes(qw)
        else:
            xv, wv, xd, wd = x, w, dev(x), dev(w)
        ref = oracle.conv2d_f64(xv, wv, (s, s), (p, p), y=y0)
        xi, wi = conv_inputs(N, C, H, W, F, KH, KW, seed=6, dist="small_int")
        exact = oracle.conv2d_f64(xi, wi, (s, s), (p, p))
        xid = dev(xi) if dt == "f32" else from_bf16_codes(oracle.bf16_encode(xi))
        wid = dev(wi) if dt == "f32" else from_bf16_codes(oracle.bf16_encode(wi))
        for cfg in tiles:
            say("direct conv", dt, cfg, case)
            y = dev(y0)
            mlk.conv2d_nchw_fchw(xd, wd, y, (s, s), (p, p), cfg=cfg)
            assert normwise(host(y), ref) <= 1e-5, (case, cfg)
            for acc in (True, False):
                y = torch.zeros(N, F, ho, wo, device="cuda") if acc else \
                    torch.full((N, F, ho, wo), float("nan"), device="cuda")
                mlk.conv2d_nchw_fchw(xid, wid, y, (s, s), (p, p), cfg=cfg, accumulate=acc)
                assert np.array_equal(host(y).astype(np.float64), exact), (case, cfg, acc)


def test_paper_conv_shape_tuned():
    """The paper's one-channel, three-filter 3x3 layer with the tile the
    exhaustive search picks (direct conv tiles included), against the oracle."""
    p = mlk.conv_problem(1, 1, 1280, 1280, 3, 3, 3, 1, 0, L.MLK_F32, L.MLK_F32)
    best, _, _ = mlk.tune(p, mlk.MLK_TUNE_EXHAUSTIVE, reps=3, warmup=1)
    assert mlk.config_legal(p, best)
    x, w = conv_inputs(1, 1, 1280, 1280, 3, 3, 3, seed=1)
    ref = oracle.conv2d_f64(x, w, threads=oracle.default_threads())
    y = torch.zeros(1, 3, 1278, 1278, device="cuda")
    mlk.conv2d_nchw_fchw(dev(x), dev(w), y, cfg=best)
    assert normwise(host(y), ref) <= 1e-5


def test_conv_call_matches_per_call_api():
    """A layer bound once (mlk.ConvCall) gives what the per-call API gives, bit
    for bit, over repeated accumulating calls, on the default and a side stream."""
    x, w = conv_inputs(2, 16, 14, 14, 32, 3, 3, seed=4)
    qx = from_bf16_codes(oracle.bf16_encode(x))
    qw = from_bf16_codes(oracle.bf16_encode(w))
    y1 = torch.zeros(2, 32, 14, 14, device="cuda")
    y2 = torch.zeros_like(y1)
    call = mlk.ConvCall(qx, qw, y1, (1, 1), (1, 1))
    side = torch.cuda.Stream()
    for k in range(3):
        if k == 1:
            torch.cuda.synchronize()
            call(stream=side)
            side.synchronize()
        else:
            call()
        mlk.conv2d_nchw_fchw(qx, qw, y2, (1, 1), (1, 1))
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
