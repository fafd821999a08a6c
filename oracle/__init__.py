"""CPU oracle for the dense kernels of arXiv 2307.16080 (nelli).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only users.  The product package never
imports this module, and this module never imports the product package.

Thin ctypes wrappers over ``liboracle.so`` (built from ``oracle.c`` by
``oracle/build.py``); numpy arrays in, numpy arrays out.  What each routine
computes, and the passage of the paper it follows, is documented in
``oracle.c``:

* matmul  -- Sec. 1, listing "nelli_for_to_affine_for"; Sec. 2.1, listing
  "linalg-matmul": C[M,N] += A[M,K] B[K,N].
* conv2d  -- Sec. 4.1, listing "2dnchwconv", with stride and zero padding.
* bf16 / OCP e4m3 encode and decode, per-tensor scale, amax.
* error statistics against a double-precision result.
* MLP forward / loss gradient / Adam (the learned cost model), in double.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double
_flt = ctypes.c_float
_vp = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "orc_matmul_f64": (None, [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _int]),
        "orc_matmul_f32": (None, [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64]),
        "orc_bias_rows_f64": (None, [_i64, _i64, _vp, _vp, _i64]),
        "orc_matmul_i8": (None, [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _int]),
        "orc_conv_out_size": (_i64, [_i64, _i64, _i64, _i64]),
        "orc_conv2d_f64": (None, [_i64] * 11 + [_vp, _vp, _vp, _int]),
        "orc_conv2d_f32": (None, [_i64] * 11 + [_vp, _vp, _vp]),
        "orc_im2col_f64": (None, [_i64] * 10 + [_vp, _vp]),
        "orc_bf16_value": (_dbl, [ctypes.c_uint16]),
        "orc_bf16_decode": (None, [_i64, _vp, _vp]),
        "orc_bf16_from_float": (ctypes.c_uint16, [_flt]),
        "orc_bf16_encode": (None, [_i64, _vp, _vp]),
        "orc_e4m3_value": (_dbl, [ctypes.c_uint8]),
        "orc_e4m3_decode": (None, [_i64, _vp, _vp]),
        "orc_e4m3_from_float": (ctypes.c_uint8, [_flt]),
        "orc_e4m3_scale": (_flt, [_flt]),
        "orc_e4m3_encode": (None, [_i64, _vp, _flt, _vp]),
        "orc_amax": (_flt, [_i64, _vp]),
        "orc_err_stats": (None, [_i64, _vp, _vp, _vp, _vp]),
        "orc_mlp_param_count": (_i64, [_i64, _i64, _i64]),
        "orc_mlp_forward": (None, [_i64, _i64, _i64, _i64, _vp, _vp, _vp]),
        "orc_mlp_loss_grad": (_dbl, [_i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp]),
        "orc_adam_step": (None, [_i64, _vp, _vp, _vp, _vp, _dbl, _dbl, _dbl, _dbl, _i64]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _c(a, dtype):
    """C-contiguous array of the given dtype (copy only when needed)."""
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


# --------------------------------------------------------------------------- matmul

def matmul_f64(A, B, C=None, threads: int = 1):
    """REF64: C + A @ B with every input converted exactly to double."""
    A = _c(A, np.float64)
    B = _c(B, np.float64)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    C = np.zeros((M, N), np.float64) if C is None else _c(C, np.float64).copy()
    _load().orc_matmul_f64(M, N, K, _p(A), K, _p(B), N, _p(C), N, threads)
    return C


def linear_f64(A, B, bias, C=None, threads: int = 1):
    """REF64 of the Linear layer (Sec. 2.1, listing "listing1"): the product A @ B
    into a zeroed buffer, then the bias nest adding bias[j] to every row; with C,
    the result is added to C (the library's accumulate mode: C += A B + bias)."""
    T = matmul_f64(A, B, threads=threads)
    M, N = T.shape
    b = _c(np.asarray(bias).reshape(-1), np.float64)
    assert b.shape[0] == N
    _load().orc_bias_rows_f64(M, N, _p(b), _p(T), N)
    if C is not None:
        T = _c(C, np.float64) + T
    return T


def matmul_f32(A, B, C=None):
    """float accumulation, product then sum each rounded (the IR's mulf/addf)."""
    A = _c(A, np.float32)
    B = _c(B, np.float32)
    M, K = A.shape
    N = B.shape[1]
    C = np.zeros((M, N), np.float32) if C is None else _c(C, np.float32).copy()
    _load().orc_matmul_f32(M, N, K, _p(A), K, _p(B), N, _p(C), N)
    return C


def matmul_i8(A, B, C=None, threads: int = 1):
    """C + sext(A) @ sext(B) with int32 wrap-around."""
    A = _c(A, np.int8)
    B = _c(B, np.int8)
    M, K = A.shape
    N = B.shape[1]
    C = np.zeros((M, N), np.int32) if C is None else _c(C, np.int32).copy()
    _load().orc_matmul_i8(M, N, K, _p(A), K, _p(B), N, _p(C), N, threads)
    return C


# --------------------------------------------------------------------------- conv

def conv_out_size(n, k, stride, pad) -> int:
    return int(_load().orc_conv_out_size(n, k, stride, pad))


def conv2d_f64(x, w, stride=(1, 1), pad=(0, 0), y=None, threads: int = 1):
    """REF64 NCHW x FCHW -> NFHW convolution (cross-correlation) with zero padding."""
    x = _c(x, np.float64)
    w = _c(w, np.float64)
    N, C, H, W = x.shape
    F, C2, KH, KW = w.shape
    assert C == C2
    sh, sw = stride
    ph, pw = pad
    HO, WO = conv_out_size(H, KH, sh, ph), conv_out_size(W, KW, sw, pw)
    y = np.zeros((N, F, HO, WO), np.float64) if y is None else _c(y, np.float64).copy()
    _load().orc_conv2d_f64(N, C, H, W, F, KH, KW, sh, sw, ph, pw, _p(x), _p(w), _p(y), threads)
    return y


def conv2d_f32(x, w, stride=(1, 1), pad=(0, 0), y=None):
    x = _c(x, np.float32)
    w = _c(w, np.float32)
    N, C, H, W = x.shape
    F, _, KH, KW = w.shape
    sh, sw = stride
    ph, pw = pad
    HO, WO = conv_out_size(H, KH, sh, ph), conv_out_size(W, KW, sw, pw)
    y = np.zeros((N, F, HO, WO), np.float32) if y is None else _c(y, np.float32).copy()
    _load().orc_conv2d_f32(N, C, H, W, F, KH, KW, sh, sw, ph, pw, _p(x), _p(w), _p(y))
    return y


def im2col_f64(x, KH, KW, stride=(1, 1), pad=(0, 0)):
    x = _c(x, np.float64)
    N, C, H, W = x.shape
    sh, sw = stride
    ph, pw = pad
    HO, WO = conv_out_size(H, KH, sh, ph), conv_out_size(W, KW, sw, pw)
    col = np.empty((C * KH * KW, N * HO * WO), np.float64)
    _load().orc_im2col_f64(N, C, H, W, KH, KW, sh, sw, ph, pw, _p(x), _p(col))
    return col


# --------------------------------------------------------------------------- formats

def bf16_encode(x):
    x = _c(x, np.float32)
    out = np.empty(x.shape, np.uint16)
    _load().orc_bf16_encode(x.size, _p(x), _p(out))
    return out


def bf16_decode(codes):
    codes = _c(codes, np.uint16)
    out = np.empty(codes.shape, np.float64)
    _load().orc_bf16_decode(codes.size, _p(codes), _p(out))
    return out


def e4m3_scale(amax: float) -> float:
    return float(_load().orc_e4m3_scale(float(amax)))


def e4m3_encode(x, scale: float):
    x = _c(x, np.float32)
    out = np.empty(x.shape, np.uint8)
    _load().orc_e4m3_encode(x.size, _p(x), float(scale), _p(out))
    return out


def e4m3_decode(codes):
    codes = _c(codes, np.uint8)
    out = np.empty(codes.shape, np.float64)
    _load().orc_e4m3_decode(codes.size, _p(codes), _p(out))
    return out


def e4m3_from_float(v: float) -> int:
    return int(_load().orc_e4m3_from_float(float(v)))


def amax(x) -> float:
    x = _c(x, np.float32)
    return float(_load().orc_amax(x.size, _p(x)))


def quantize_e4m3(x):
    """Per-tensor scaling: returns (codes, scale) with scale = amax/448."""
    s = e4m3_scale(amax(x))
    return e4m3_encode(x, s), s


# --------------------------------------------------------------------------- errors

def err_stats(c, r, bound=None):
    """(sum (c-r)^2, sum r^2, max|c-r|, max |c-r|/bound) in double."""
    c = _c(c, np.float64).ravel()
    r = _c(r, np.float64).ravel()
    out = np.zeros(4, np.float64)
    bp = None
    if bound is not None:
        bound = _c(bound, np.float64).ravel()
        bp = _p(bound)
    _load().orc_err_stats(c.size, _p(c), _p(r), bp, _p(out))
    return out


def normwise_rel_err(c, r) -> float:
    s = err_stats(c, r)
    return float(np.sqrt(s[0] / s[1])) if s[1] > 0 else float(np.sqrt(s[0]))


# --------------------------------------------------------------------------- MLP

def mlp_param_count(D0, H1, H2) -> int:
    return int(_load().orc_mlp_param_count(D0, H1, H2))


def mlp_forward(p, X, H1, H2):
    X = _c(X, np.float64)
    p = _c(p, np.float64)
    B, D0 = X.shape
    y = np.empty(B, np.float64)
    _load().orc_mlp_forward(B, D0, H1, H2, _p(p), _p(X), _p(y))
    return y


def mlp_loss_grad(p, X, t, H1, H2):
    X = _c(X, np.float64)
    p = _c(p, np.float64)
    t = _c(t, np.float64)
    B, D0 = X.shape
    g = np.empty_like(p)
    loss = _load().orc_mlp_loss_grad(B, D0, H1, H2, _p(p), _p(X), _p(t), _p(g))
    return float(loss), g


def adam_step(p, g, m, v, lr, b1, b2, eps, t):
    """In place on p, m, v (float64 contiguous arrays)."""
    for a in (p, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _load().orc_adam_step(p.size, _p(p), _p(g), _p(m), _p(v), lr, b1, b2, eps, t)
