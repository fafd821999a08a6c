"""MI355X (gfx950) dense kernels for the computations of arXiv 2307.16080 (nelli).

Thin Python binding over the C ABI of ``libmlk.so`` (``include/mlk.h``): it
marshals torch tensors (device memory and streams only) into plain pointers
and sizes.  Every step of every operation runs in the library's HIP kernels;
there is no CPU or PyTorch fallback.

    matmul(A, B, C)                 C (+)= A @ B          (linalg.matmul)
    conv2d_nchw_fchw(x, w, y, ...)  y (+)= conv(x, w)      (linalg.conv_2d_nchw_fchw)
    quantize(x, "bf16" | "e4m3")    per-tensor quantisation for the low-precision paths
    batched_matmul([...])           many uneven GEMMs, optionally one persistent launch / graph
    err_stats(c, r, bound)          FP64 error reduction against a double reference
    tune(problem, ...)              tile-configuration search (exhaustive / random / model)
    CostModel                       the learned cost model (MLP trained on the GPU)
"""
import ctypes

import torch

from . import _lib as L
from ._lib import (MLK_BATCH_GRAPH, MLK_BATCH_PERSISTENT, MLK_BF16, MLK_F8E4M3, MLK_F32, MLK_I8,
                   MLK_I32, MLK_OP_BATCHED, MLK_OP_CONV2D, MLK_OP_MATMUL, MLK_TUNE_EXHAUSTIVE,
                   MLK_TUNE_ES, MLK_TUNE_MODEL, MLK_TUNE_RANDOM, GemmDesc, MlkError, Problem, TileConfig,
                   TuneOpts, TuneReport)

__all__ = ["matmul", "matmul_noalloc", "matmul_bias", "conv2d_nchw_fchw", "ConvCall", "ConvBatch", "quantize", "batched_matmul", "BatchedCall", "err_stats", "tune",
           "config_count", "configs", "config_legal", "mfma_rate", "set_default_config", "CostModel",
           "mlp_forward", "mlp_loss_grad", "adam_step", "release", "version", "TileConfig",
           "Problem", "MlkError", "matmul_problem", "conv_problem", "batched_problem"]

_TORCH_TO_MLK = {
    torch.float32: MLK_F32,
    torch.bfloat16: MLK_BF16,
    torch.float8_e4m3fn: MLK_F8E4M3,
    torch.int8: MLK_I8,
    torch.int32: MLK_I32,
}


def _dt(t: torch.Tensor) -> int:
    try:
        return _TORCH_TO_MLK[t.dtype]
    except KeyError:
        raise MlkError(4, f"unsupported tensor dtype {t.dtype}") from None


def _on_device(t):
    """The library takes device memory only: a host tensor is refused here,
    before its address could reach a kernel."""
    if isinstance(t, torch.Tensor) and not t.is_cuda:
        raise MlkError(9, f"expected a tensor in GPU memory, got one on {t.device}")
    return t


def _need(cond, status, msg):
    if not cond:
        raise MlkError(status, msg)


def _check_scale(t, what):
    if t is not None:
        _need(isinstance(t, torch.Tensor) and t.dtype == torch.float32 and t.numel() >= 1, 9,
              f"{what} must be a float32 tensor of at least one element")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(_on_device(t).data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _cfg(cfg):
    if cfg is None:
        return None
    if isinstance(cfg, TileConfig):
        return ctypes.byref(cfg)
    return ctypes.byref(TileConfig(*cfg))


def _row_major_ld(t: torch.Tensor) -> int:
    if t.dim() != 2 or t.stride(1) != 1:
        raise MlkError(3, "expected a 2-D tensor with unit column stride (row-major)")
    return t.stride(0) if t.size(0) > 1 else max(t.size(1), 1)


def version() -> str:
    return L.lib().mlk_version().decode()


def release() -> None:
    L.lib().mlk_release()


# --------------------------------------------------------------------------- matmul / conv

def matmul(A, B, C, accumulate: bool = True, cfg=None, scale_a=None, scale_b=None, stream=None):
    """C (+)= A @ B.  A: (M, K), B: (K, N), C: (M, N), row-major CUDA tensors.

    (float32, float32), (bfloat16, float32), (float8_e4m3fn, float32) with optional
    device scale tensors, (int8, int32); bfloat16 C with bfloat16 or float8_e4m3fn
    inputs (the fp32 result rounded once to bf16; split_k 1)."""
    _need(A.dim() == 2 and B.dim() == 2 and C.dim() == 2, 2, "matmul operands must be 2-D")
    M, K = A.shape
    K2, N = B.shape
    if K2 != K or tuple(C.shape) != (M, N):
        raise MlkError(2, f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}, C {tuple(C.shape)}")
    _need(B.dtype == A.dtype, 4, f"A and B must have one dtype (got {A.dtype}, {B.dtype})")
    _check_scale(scale_a, "scale_a")
    _check_scale(scale_b, "scale_b")
    L.check(L.lib().mlk_matmul(_dt(A), _dt(C), M, N, K, _ptr(A), _row_major_ld(A), _ptr(B),
                               _row_major_ld(B), _ptr(C), _row_major_ld(C), _ptr(scale_a),
                               _ptr(scale_b), int(bool(accumulate)), _cfg(cfg), _stream(stream)))
    return C


def matmul_noalloc(A, B, C, accumulate: bool = True, cfg=None, scale_a=None, scale_b=None, stream=None):
    """matmul through mlk_matmul_noalloc: operand packing (when the tile needs it)
    uses the library's fixed per-device array, so the call allocates nothing
    (usable under graph capture).  Calls overlapping on one device race on it."""
    _need(A.dim() == 2 and B.dim() == 2 and C.dim() == 2, 2, "matmul operands must be 2-D")
    M, K = A.shape
    K2, N = B.shape
    if K2 != K or tuple(C.shape) != (M, N):
        raise MlkError(2, f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}, C {tuple(C.shape)}")
    _need(B.dtype == A.dtype, 4, f"A and B must have one dtype (got {A.dtype}, {B.dtype})")
    _check_scale(scale_a, "scale_a")
    _check_scale(scale_b, "scale_b")
    L.check(L.lib().mlk_matmul_noalloc(_dt(A), _dt(C), M, N, K, _ptr(A), _row_major_ld(A), _ptr(B),
                                       _row_major_ld(B), _ptr(C), _row_major_ld(C), _ptr(scale_a),
                                       _ptr(scale_b), int(bool(accumulate)), _cfg(cfg), _stream(stream)))
    return C


def matmul_bias(A, B, bias, C, accumulate: bool = False, cfg=None, scale_a=None, scale_b=None,
                stream=None):
    """The Linear layer: C (+)= A @ B + bias, the bias add fused into the product's output.

    bias: float32 CUDA tensor of N elements.  Float outputs only (the float pairs of matmul)."""
    _need(A.dim() == 2 and B.dim() == 2 and C.dim() == 2, 2, "matmul operands must be 2-D")
    M, K = A.shape
    K2, N = B.shape
    if K2 != K or tuple(C.shape) != (M, N):
        raise MlkError(2, f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}, C {tuple(C.shape)}")
    _need(B.dtype == A.dtype, 4, f"A and B must have one dtype (got {A.dtype}, {B.dtype})")
    _check_scale(scale_a, "scale_a")
    _check_scale(scale_b, "scale_b")
    if bias.dtype != torch.float32 or bias.numel() != N or not bias.is_contiguous():
        raise MlkError(2, f"bias must be {N} contiguous float32 values")
    L.check(L.lib().mlk_matmul_bias(_dt(A), _dt(C), M, N, K, _ptr(A), _row_major_ld(A), _ptr(B),
                                    _row_major_ld(B), _ptr(bias), _ptr(C), _row_major_ld(C),
                                    _ptr(scale_a), _ptr(scale_b), int(bool(accumulate)), _cfg(cfg),
                                    _stream(stream)))
    return C


def _conv_args(x, w, y, stride, pad, accumulate):
    """Checked arguments of mlk_conv2d_nchw_fchw up to (not including) cfg and stream."""
    for t in (x, w, y):
        if not t.is_contiguous():
            raise MlkError(3, "conv2d tensors must be contiguous")
    _need(x.dim() == 4 and w.dim() == 4 and y.dim() == 4, 2, "conv2d tensors must be 4-D")
    N, C, H, W = x.shape
    F, C2, KH, KW = w.shape
    if C2 != C:
        raise MlkError(2, "channel mismatch")
    _need(w.dtype == x.dtype, 4, f"x and w must have one dtype (got {x.dtype}, {w.dtype})")
    sh, sw = stride
    ph, pw = pad
    if sh > 0 and sw > 0:
        HO, WO = conv_out_hw(H, W, KH, KW, stride, pad)
        if HO > 0 and WO > 0:
            _need(tuple(y.shape) == (N, F, HO, WO), 2,
                  f"y must be {(N, F, HO, WO)} for these inputs, got {tuple(y.shape)}")
    return (_dt(x), _dt(y), N, C, H, W, F, KH, KW, sh, sw, ph, pw, _ptr(x), _ptr(w), _ptr(y),
            int(bool(accumulate)))


def conv2d_nchw_fchw(x, w, y, stride=(1, 1), pad=(0, 0), accumulate: bool = True, cfg=None,
                     stream=None):
    """y (+)= conv(x, w): x (N,C,H,W), w (F,C,KH,KW), y (N,F,HO,WO), contiguous."""
    L.check(L.lib().mlk_conv2d_nchw_fchw(*_conv_args(x, w, y, stride, pad, accumulate), _cfg(cfg),
                                         _stream(stream)))
    return y


class ConvCall:
    """One convolution bound once to its tensors (mlk_conv2d_plan_*): shape,
    configuration and filter are checked, resolved and bound here, so each
    call is a single library call that allocates nothing and may be recorded
    into a captured graph.  The filter's values are those at binding (or at
    the last update_filter()).  The tensors are kept alive by the object; their
    storage must not move between calls.  `stream`, if given here, orders the
    binding's own work (the filter transpose of the channels-last and channel-gather layouts) and is the default
    for every call."""

    def __init__(self, x, w, y, stride=(1, 1), pad=(0, 0), accumulate: bool = True, cfg=None,
                 stream=None):
        a = _conv_args(x, w, y, stride, pad, accumulate)
        self._keep = (x, w, y)
        self._cfg = None if cfg is None else (cfg if isinstance(cfg, TileConfig) else TileConfig(*cfg))
        self._stream = None if stream is None else _stream(stream)
        h = ctypes.c_void_p()
        # (din, dout, N, C, H, W, F, KH, KW, sh, sw, ph, pw, x, w, y, accumulate)
        L.check(L.lib().mlk_conv2d_plan_create(*a[:13], a[14], a[16], _cfg(self._cfg),
                                               self._stream if self._stream is not None else _stream(None),
                                               ctypes.byref(h)))
        self._plan = h.value
        self._x, self._y = a[13], a[15]
        self._run = L.lib().mlk_conv2d_plan_run

    @property
    def config(self):
        c = TileConfig()
        L.check(L.lib().mlk_conv2d_plan_config(self._plan, ctypes.byref(c)))
        return c

    def update_filter(self, stream=None):
        L.check(L.lib().mlk_conv2d_plan_update_filter(self._plan, _stream(stream) if stream is not None
                                                      else (self._stream or _stream(None))))

    def __call__(self, stream=None):
        if stream is not None:
            st = _stream(stream)
        else:
            st = self._stream if self._stream is not None else _stream(None)
        L.check(self._run(self._plan, self._x, self._y, st))
        return self._keep[2]

    def __del__(self):
        if getattr(self, "_plan", None) and L._lib is not None:
            L.lib().mlk_conv2d_plan_destroy(self._plan)
            self._plan = None


class ConvBatch:
    """Many independent convolutions in one persistent launch (mlk_conv2d_batch_*):
    a list of (x, w, y, stride, pad) with x, w bfloat16 NCHW / FCHW and y float32
    NFHW, all contiguous CUDA tensors, C a multiple of 8.  The tensors are bound
    at creation (their storage must not move); each call runs every convolution,
    y (+)= conv(x, w), as one launch (plus, when overwriting, a zero fill of each
    split output), allocates nothing and may be captured into a graph.  `cfg`:
    None (64 x 64 tile, split cap 16) or a register-loaded conv tile with
    stages 1, layout 3 and split_k = the largest K split per convolution."""

    def __init__(self, convs, accumulate: bool = True, cfg=None, stream=None):
        descs = (L.ConvDesc * len(convs))()
        keep = []
        for i, (x, w, y, stride, pad) in enumerate(convs):
            for t in (x, w, y):
                _need(t.is_contiguous(), 3, "conv batch tensors must be contiguous")
                _on_device(t)
            _need(x.dim() == 4 and w.dim() == 4 and y.dim() == 4, 2, "conv batch tensors must be 4-D")
            _need(x.dtype == torch.bfloat16 and w.dtype == torch.bfloat16 and y.dtype == torch.float32, 4,
                  "conv batch: bfloat16 x and w, float32 y")
            N, C, H, W = x.shape
            F, C2, KH, KW = w.shape
            _need(C2 == C, 2, f"conv batch: channel mismatch in convolution {i}")
            ho, wo = conv_out_hw(H, W, KH, KW, stride, pad)
            _need(tuple(y.shape) == (N, F, ho, wo), 2, f"conv batch: y of convolution {i} must be {(N, F, ho, wo)}")
            descs[i] = L.ConvDesc(N, C, H, W, F, KH, KW, stride[0], stride[1], pad[0], pad[1], x.data_ptr(),
                                  w.data_ptr(), y.data_ptr())
            keep.append((x, w, y))
        self._keep = keep
        self._stream = None if stream is None else _stream(stream)
        h = ctypes.c_void_p()
        cfg_ = None if cfg is None else (cfg if isinstance(cfg, TileConfig) else TileConfig(*cfg))
        L.check(L.lib().mlk_conv2d_batch_create(MLK_BF16, MLK_F32, len(convs), descs, int(bool(accumulate)),
                                                _cfg(cfg_), self._stream if self._stream is not None else
                                                _stream(None), ctypes.byref(h)))
        self._batch = h.value

    def info(self):
        """(TileConfig, tasks, workgroups) of the planned launch."""
        c, t, w = TileConfig(), ctypes.c_int64(), ctypes.c_int32()
        L.check(L.lib().mlk_conv2d_batch_info(self._batch, ctypes.byref(c), ctypes.byref(t), ctypes.byref(w)))
        return c, t.value, w.value

    def update_filters(self, stream=None):
        L.check(L.lib().mlk_conv2d_batch_update_filters(
            self._batch, _stream(stream) if stream is not None else (self._stream or _stream(None))))

    def __call__(self, stream=None):
        st = _stream(stream) if stream is not None else (self._stream if self._stream is not None else _stream(None))
        L.check(L.lib().mlk_conv2d_batch_run(self._batch, st))
        return [y for _, _, y in self._keep]

    def __del__(self):
        if getattr(self, "_batch", None) and L._lib is not None:
            L.lib().mlk_conv2d_batch_destroy(self._batch)
            self._batch = None


def mfma_rate(dtype="bf16", iters=4096, stream=None):
    """Launch the MFMA rate probe once (mlk_mfma_rate): returns (flops of the
    launch, the per-wave float32 results, each exactly 28 + 8 * iters * k)."""
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    out = torch.empty(8 * props.multi_processor_count, dtype=torch.float32, device="cuda")
    flops = ctypes.c_int64()
    L.check(L.lib().mlk_mfma_rate({"bf16": MLK_BF16, "e4m3": MLK_F8E4M3}[dtype], int(iters), _ptr(out), out.numel(),
                                  ctypes.byref(flops), _stream(stream)))
    return flops.value, out


def conv_out_hw(H, W, KH, KW, stride=(1, 1), pad=(0, 0)):
    return ((H + 2 * pad[0] - KH) // stride[0] + 1, (W + 2 * pad[1] - KW) // stride[1] + 1)


def quantize(x: torch.Tensor, fmt: str, q=None, scale=None, stream=None):
    """Quantise a float32 CUDA tensor.  fmt "bf16" -> (q, None); "e4m3" -> (q, scale)
    with scale a one-element float32 device tensor (amax / 448)."""
    if x.dtype != torch.float32 or not x.is_contiguous():
        raise MlkError(4, "quantize expects a contiguous float32 tensor")
    def _out(t, dtype):
        _need(t.dtype == dtype and t.is_contiguous() and t.numel() >= x.numel(), 2,
              f"q must be a contiguous {dtype} tensor of at least {x.numel()} elements")
    if fmt == "bf16":
        q = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device) if q is None else q
        _out(q, torch.bfloat16)
        L.check(L.lib().mlk_quantize(MLK_BF16, x.numel(), _ptr(x), _ptr(q), None, _stream(stream)))
        return q, None
    if fmt == "e4m3":
        q = torch.empty(x.shape, dtype=torch.float8_e4m3fn, device=x.device) if q is None else q
        scale = torch.empty(1, dtype=torch.float32, device=x.device) if scale is None else scale
        _out(q, torch.float8_e4m3fn)
        _check_scale(scale, "scale")
        L.check(L.lib().mlk_quantize(MLK_F8E4M3, x.numel(), _ptr(x), _ptr(q), _ptr(scale),
                                     _stream(stream)))
        return q, scale
    raise MlkError(4, f"unknown format {fmt!r}")


class BatchedCall:
    """A batch of GEMMs bound once to its tensors.  The descriptor array is built
    here, once; each call is then a single library call (with `graph`, a replay
    of the captured launches), so a serving loop pays no per-GEMM host work.
    cfg: None (the batch's tuned choice, else the heuristic), one TileConfig for
    every GEMM, or a list of one per GEMM (None entries: that GEMM chooses).
    The tensors are kept alive by the object; their storage must not move
    between calls."""

    def __init__(self, problems, accumulate: bool = True, cfg=None, persistent: bool = False,
                 graph: bool = False):
        if len(problems) == 0:
            raise MlkError(2, "batched: empty problem list")
        self._problems = list(problems)
        self._descs = (GemmDesc * len(self._problems))()
        A0, B0, C0 = self._problems[0]
        for i, (A, B, C) in enumerate(self._problems):
            _need(A.dim() == 2 and B.dim() == 2 and C.dim() == 2, 2, f"batched: GEMM {i}: operands must be 2-D")
            _need(B.shape[0] == A.shape[1] and tuple(C.shape) == (A.shape[0], B.shape[1]), 2,
                  f"batched: GEMM {i}: shapes A {tuple(A.shape)}, B {tuple(B.shape)}, C {tuple(C.shape)}")
            _need(A.dtype == A0.dtype and B.dtype == A0.dtype and C.dtype == C0.dtype, 4,
                  f"batched: GEMM {i}: every A and B must be {A0.dtype} and every C {C0.dtype}")
        for i, (A, B, C) in enumerate(self._problems):
            M, K = A.shape
            N = B.shape[1]
            self._descs[i] = GemmDesc(M, N, K, _on_device(A).data_ptr(), _row_major_ld(A),
                                      _on_device(B).data_ptr(), _row_major_ld(B), _on_device(C).data_ptr(),
                                      _row_major_ld(C))
        self._din, self._dout = _dt(A0), _dt(C0)
        if cfg is None:
            self._cfgs, self._ncfgs = None, 0
        elif isinstance(cfg, list):
            _need(len(cfg) == len(self._problems), 9,
                  f"batched: {len(cfg)} configurations for {len(self._problems)} GEMMs")
            self._cfgs = (TileConfig * len(cfg))(*[TileConfig() if c is None else
                                                   (c if isinstance(c, TileConfig) else TileConfig(*c)) for c in cfg])
            self._ncfgs = len(cfg)
        else:
            self._cfgs = (TileConfig * 1)(cfg if isinstance(cfg, TileConfig) else TileConfig(*cfg))
            self._ncfgs = 1
        self._acc = int(bool(accumulate))
        self._flags = (MLK_BATCH_PERSISTENT if persistent else 0) | (MLK_BATCH_GRAPH if graph else 0)

    def __call__(self, stream=None):
        L.check(L.lib().mlk_batched_matmul(self._din, self._dout, len(self._problems), self._descs,
                                           self._cfgs, self._ncfgs, self._acc, self._flags, _stream(stream)))


def batched_matmul(problems, accumulate: bool = True, cfg=None, persistent: bool = False,
                   graph: bool = False, stream=None):
    """problems: list of (A, B, C) CUDA tensors (same dtypes across the list).
    cfg: None, one TileConfig for all, or a list with one per GEMM."""
    BatchedCall(problems, accumulate, cfg, persistent, graph)(stream)


def err_stats(c: torch.Tensor, r: torch.Tensor, bound=None, stream=None):
    """(sum (c-r)^2, sum r^2, max|c-r|, max |c-r|/bound) reduced on the GPU in FP64."""
    out = torch.empty(4, dtype=torch.float64, device=c.device)
    if r.dtype != torch.float64 or (bound is not None and bound.dtype != torch.float64):
        raise MlkError(4, "reference and bound must be float64")
    _need(c.is_contiguous() and r.is_contiguous() and r.numel() == c.numel() and
          (bound is None or (bound.is_contiguous() and bound.numel() == c.numel())), 2,
          "err_stats: c, r (and bound) must be contiguous with one element count")
    L.check(L.lib().mlk_err_stats(_dt(c), c.numel(), _ptr(c), _ptr(r), _ptr(bound), _ptr(out),
                                  _stream(stream)))
    return out


# --------------------------------------------------------------------------- tuning

def matmul_problem(M, N, K, in_dtype=MLK_BF16, out_dtype=MLK_F32, accumulate=True):
    p = Problem()
    p.op, p.in_, p.out, p.accumulate = MLK_OP_MATMUL, in_dtype, out_dtype, int(bool(accumulate))
    p.M, p.N, p.K = M, N, K
    return p


def conv_problem(n, c, h, w, f, kh, kw, stride=1, pad=0, in_dtype=MLK_BF16, out_dtype=MLK_F32,
                 accumulate=True):
    p = Problem()
    p.op, p.in_, p.out, p.accumulate = MLK_OP_CONV2D, in_dtype, out_dtype, int(bool(accumulate))
    p.n, p.c, p.h, p.w, p.f, p.kh, p.kw = n, c, h, w, f, kh, kw
    p.sh = p.sw = stride
    p.ph = p.pw = pad
    return p


def batched_problem(shapes, in_dtype=MLK_BF16, out_dtype=MLK_F32, accumulate=True):
    """shapes: list of (M, N, K).  The descriptor array is kept alive on the problem."""
    descs = (GemmDesc * len(shapes))()
    for i, (M, N, K) in enumerate(shapes):
        descs[i] = GemmDesc(M, N, K, None, max(K, 1), None, max(N, 1), None, max(N, 1))
    p = Problem()
    p.op, p.in_, p.out, p.accumulate = MLK_OP_BATCHED, in_dtype, out_dtype, int(bool(accumulate))
    p.count = len(shapes)
    p.descs = ctypes.cast(descs, ctypes.POINTER(GemmDesc))
    p._keep = descs
    return p


def config_count(problem) -> int:
    n = L.lib().mlk_config_count(ctypes.byref(problem))
    if n < 0:
        L.check(L.lib().mlk_config_legal(ctypes.byref(problem), ctypes.byref(TileConfig())))
    return n


def configs(problem):
    out = []
    for i in range(config_count(problem)):
        c = TileConfig()
        L.check(L.lib().mlk_config_get(ctypes.byref(problem), i, ctypes.byref(c)))
        out.append(c)
    return out


def config_legal(problem, cfg) -> bool:
    return L.lib().mlk_config_legal(ctypes.byref(problem), _cfg(cfg)) == 0


def set_default_config(problem, cfg):
    L.check(L.lib().mlk_config_set_default(ctypes.byref(problem), _cfg(cfg)))


def tune(problem, strategy=MLK_TUNE_EXHAUSTIVE, budget_frac=1.0, reps=0, warmup=0, seed=0,
         db_path=None, use_db=False, model=None, want_times=False, fake_timer=False, table=None):
    """Returns (best TileConfig, TuneReport, times_us list or None).  `table`: one time per
    legal configuration (enumeration order) to replay the search on instead of measuring."""
    n = config_count(problem)
    times = (ctypes.c_double * max(n, 1))() if want_times else None
    tab = None
    if table is not None:
        if len(table) != n:
            raise MlkError(9, f"tune: table has {len(table)} entries for {n} configurations")
        tab = (ctypes.c_double * n)(*[float(v) for v in table])
    o = TuneOpts()
    o.strategy, o.budget_frac, o.reps, o.warmup, o.seed = strategy, budget_frac, reps, warmup, seed
    o.db_path = db_path.encode() if db_path else None
    o.use_db = int(bool(use_db))
    o.model = model.handle if model is not None else None
    o.times_us = ctypes.cast(times, ctypes.POINTER(ctypes.c_double)) if times is not None else None
    o.fake_timer = int(bool(fake_timer))
    o.table_us = ctypes.cast(tab, ctypes.POINTER(ctypes.c_double)) if tab is not None else None
    best, rep = TileConfig(), TuneReport()
    L.check(L.lib().mlk_tune(ctypes.byref(problem), ctypes.byref(o), ctypes.byref(best),
                             ctypes.byref(rep)))
    return best, rep, (list(times)[:n] if times is not None else None)


class CostModel:
    """The learned cost model (owns device buffers inside the library)."""

    def __init__(self, hidden=64, seed=0):
        h = ctypes.c_void_p()
        L.check(L.lib().mlk_model_create(hidden, seed, ctypes.byref(h)))
        self.handle = h.value

    def __del__(self):
        if getattr(self, "handle", None) and L._lib is not None:
            L.lib().mlk_model_destroy(self.handle)
            self.handle = None

    def add_sample(self, problem, cfg, time_us):
        L.check(L.lib().mlk_model_add_sample(self.handle, ctypes.byref(problem), _cfg(cfg), time_us))

    def sample_count(self):
        return L.lib().mlk_model_sample_count(self.handle)

    def train(self, epochs=200, batch=256, lr=1e-3):
        loss = ctypes.c_float()
        L.check(L.lib().mlk_model_train(self.handle, epochs, batch, lr, ctypes.byref(loss)))
        return loss.value

    def predict(self, problem, cfgs):
        arr = (TileConfig * len(cfgs))(*cfgs)
        out = (ctypes.c_float * len(cfgs))()
        L.check(L.lib().mlk_model_predict(self.handle, ctypes.byref(problem), arr, len(cfgs), out))
        return list(out)


def features(problem, cfg):
    n = L.lib().mlk_model_feature_count()
    out = (ctypes.c_float * n)()
    L.check(L.lib().mlk_model_features(ctypes.byref(problem), _cfg(cfg), out))
    return list(out)


# --------------------------------------------------------------------------- cost-model kernels

def mlp_param_count(D0, H1, H2):
    """Length of the flat parameter vector: W1, b1, W2, b2, W3, b3."""
    return D0 * H1 + H1 + H1 * H2 + H2 + H2 + 1


def _check_mlp(params, X, H1, H2):
    _need(X.dim() == 2 and X.dtype == torch.float32 and X.is_contiguous(), 2, "X must be a contiguous 2-D float32 tensor")
    _need(params.dtype == torch.float32 and params.is_contiguous() and
          params.numel() == mlp_param_count(X.shape[1], H1, H2), 2,
          f"params must hold {mlp_param_count(X.shape[1], H1, H2)} contiguous float32 values")


def mlp_forward(params, X, H1, H2, stream=None):
    _check_mlp(params, X, H1, H2)
    B, D0 = X.shape
    y = torch.empty(B, dtype=torch.float32, device=X.device)
    L.check(L.lib().mlk_mlp_forward(B, D0, H1, H2, _ptr(params), _ptr(X), _ptr(y), _stream(stream)))
    return y


def mlp_loss_grad(params, X, t, H1, H2, stream=None):
    _check_mlp(params, X, H1, H2)
    _need(t.dtype == torch.float32 and t.is_contiguous() and t.numel() == X.shape[0], 2,
          "t must hold one contiguous float32 target per row of X")
    B, D0 = X.shape
    g = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    L.check(L.lib().mlk_mlp_loss_grad(B, D0, H1, H2, _ptr(params), _ptr(X), _ptr(t), _ptr(g),
                                      _ptr(loss), _stream(stream)))
    return loss, g


def adam_step(params, grad, m, v, lr, beta1, beta2, eps, t, stream=None):
    for a in (params, grad, m, v):
        _need(a.dtype == torch.float32 and a.is_contiguous() and a.numel() == params.numel(), 2,
              "adam_step: params, grad, m and v must be contiguous float32 tensors of one length")
    L.check(L.lib().mlk_adam_step(params.numel(), _ptr(params), _ptr(grad), _ptr(m), _ptr(v), lr,
                                  beta1, beta2, eps, t, _stream(stream)))
