"""Binding of the OpenMP host kernels (``libmlkhost.so``, ``include/mlk_host.h``):
the paper's CPU lowering of matmul and conv2d with a searched tiling and unroll
factor.  Host numpy arrays in, results written in place; argument marshalling
only.  This is a separate library: nothing in the GPU package calls it.

    matmul_f32(A, B, C, accumulate=True, cfg=None)
    conv2d_f32(x, w, y, stride, pad, accumulate=True, cfg=None)
    tune("matmul", (M, N, K)) / tune("conv", (N, C, H, W, F, KH, KW, sh, sw, ph, pw))
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlkhost.so")


class HostConfig(ctypes.Structure):
    _fields_ = [("mb", ctypes.c_int32), ("nb", ctypes.c_int32), ("kb", ctypes.c_int32),
                ("unroll", ctypes.c_int32), ("threads", ctypes.c_int32)]

    def as_tuple(self):
        return tuple(getattr(self, f) for f, _ in self._fields_)

    def __repr__(self):
        return "HostConfig(%s)" % ", ".join(f"{f}={getattr(self, f)}" for f, _ in self._fields_)


_i32, _i64, _vp, _int = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
_cfgp = ctypes.POINTER(HostConfig)
_dimsp = ctypes.POINTER(ctypes.c_int64)
SIGNATURES = {
    "mlkh_matmul_f32": (_int, [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _int, _cfgp]),
    "mlkh_conv2d_f32": (_int, [_i64, _i64, _i64, _i64, _i64, _i64, _i64, _i32, _i32, _i32, _i32, _vp, _vp, _vp,
                               _int, _cfgp]),
    "mlkh_config_count": (_i32, [_i32, _dimsp]),
    "mlkh_config_get": (_int, [_i32, _dimsp, _i32, _cfgp]),
    "mlkh_tune": (_int, [_i32, _dimsp, _i32, ctypes.c_double, _i32, ctypes.c_uint64, _cfgp,
                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "mlkh_max_threads": (_i32, []),
}
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2307_16080_amd.build`")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype, fn.argtypes = res, args
        _lib = h
    return _lib


def _check(st):
    if st != 0:
        raise RuntimeError(f"mlk host kernel returned status {st}")


def _f32(a, name):
    if not (isinstance(a, np.ndarray) and a.dtype == np.float32 and a.flags["C_CONTIGUOUS"]):
        raise TypeError(f"{name} must be a C-contiguous float32 numpy array")
    return a.ctypes.data_as(ctypes.c_void_p)


def _cfg(cfg):
    if cfg is None:
        return None
    return ctypes.byref(cfg if isinstance(cfg, HostConfig) else HostConfig(*cfg))


def matmul_f32(A, B, C, accumulate=True, cfg=None):
    M, K = A.shape
    K2, N = B.shape
    if K2 != K or C.shape != (M, N):
        raise ValueError(f"shape mismatch: A {A.shape}, B {B.shape}, C {C.shape}")
    _check(lib().mlkh_matmul_f32(M, N, K, _f32(A, "A"), K, _f32(B, "B"), N, _f32(C, "C"), N, int(bool(accumulate)),
                                 _cfg(cfg)))
    return C


def conv2d_f32(x, w, y, stride=(1, 1), pad=(0, 0), accumulate=True, cfg=None):
    N, C, H, W = x.shape
    F, C2, KH, KW = w.shape
    HO, WO = (H + 2 * pad[0] - KH) // stride[0] + 1, (W + 2 * pad[1] - KW) // stride[1] + 1
    if C2 != C or y.shape != (N, F, HO, WO):
        raise ValueError(f"shape mismatch: x {x.shape}, w {w.shape}, y {y.shape}")
    _check(lib().mlkh_conv2d_f32(N, C, H, W, F, KH, KW, stride[0], stride[1], pad[0], pad[1], _f32(x, "x"),
                                 _f32(w, "w"), _f32(y, "y"), int(bool(accumulate)), _cfg(cfg)))
    return y


def _op_dims(kind, dims):
    op = {"matmul": 0, "conv": 1}[kind]
    d = (ctypes.c_int64 * 11)(*([int(v) for v in dims] + [0] * (11 - len(dims))))
    return op, d


def configs(kind, dims):
    op, d = _op_dims(kind, dims)
    n = lib().mlkh_config_count(op, d)
    out = []
    for i in range(n):
        c = HostConfig()
        _check(lib().mlkh_config_get(op, d, i, ctypes.byref(c)))
        out.append(c)
    return out


def tune(kind, dims, strategy=0, budget_frac=1.0, reps=5, seed=0, want_times=False):
    """strategy 0: every configuration; 1: (1+1) evolution strategy within the budget.
    Returns (best HostConfig, its median microseconds, times per configuration or None)."""
    op, d = _op_dims(kind, dims)
    n = lib().mlkh_config_count(op, d)
    times = (ctypes.c_double * max(n, 1))() if want_times else None
    best, us = HostConfig(), ctypes.c_double()
    _check(lib().mlkh_tune(op, d, strategy, budget_frac, reps, seed, ctypes.byref(best), ctypes.byref(us),
                           ctypes.cast(times, ctypes.POINTER(ctypes.c_double)) if times is not None else None))
    return best, us.value, (list(times)[:n] if times is not None else None)


def max_threads():
    return lib().mlkh_max_threads()
