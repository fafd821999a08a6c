"""ctypes declarations of the C ABI in ``include/mlk.h`` (argument marshalling only).

``torch`` is imported first so that its HIP runtime (``libamdhip64.so.7``) is the
one the library binds to: device pointers and streams then come from one
runtime.  A missing ``libmlk.so`` is an error, never a fallback.
"""
import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library links against)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlk.so")

# status codes
MLK_OK = 0
STATUS_NAMES = ["MLK_OK", "MLK_ERR_NULL", "MLK_ERR_SHAPE", "MLK_ERR_LAYOUT", "MLK_ERR_DTYPE",
                "MLK_ERR_CONFIG", "MLK_ERR_DB", "MLK_ERR_HIP", "MLK_ERR_NOMEM", "MLK_ERR_ARG"]
# dtypes
MLK_F32, MLK_BF16, MLK_F8E4M3, MLK_I8, MLK_I32 = 0, 1, 2, 3, 4
# ops / strategies / flags
MLK_OP_MATMUL, MLK_OP_CONV2D, MLK_OP_BATCHED = 0, 1, 2
MLK_TUNE_EXHAUSTIVE, MLK_TUNE_RANDOM, MLK_TUNE_MODEL, MLK_TUNE_ES = 0, 1, 2, 3
MLK_BATCH_PERSISTENT, MLK_BATCH_GRAPH = 1, 2


class TileConfig(ctypes.Structure):
    _fields_ = [("bm", ctypes.c_int32), ("bn", ctypes.c_int32), ("bk", ctypes.c_int32),
                ("wm", ctypes.c_int32), ("wn", ctypes.c_int32), ("split_k", ctypes.c_int32),
                ("group_m", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("stages", ctypes.c_int32), ("layout", ctypes.c_int32), ("mfma", ctypes.c_int32)]

    def as_tuple(self):
        return tuple(getattr(self, f) for f, _ in self._fields_)

    def __repr__(self):
        return "TileConfig(%s)" % ", ".join(f"{f}={getattr(self, f)}" for f, _ in self._fields_)


class GemmDesc(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64)]


class ConvDesc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("C", ctypes.c_int64), ("H", ctypes.c_int64), ("W", ctypes.c_int64),
                ("F", ctypes.c_int64), ("KH", ctypes.c_int64), ("KW", ctypes.c_int64),
                ("sh", ctypes.c_int32), ("sw", ctypes.c_int32), ("ph", ctypes.c_int32), ("pw", ctypes.c_int32),
                ("x", ctypes.c_void_p), ("w", ctypes.c_void_p), ("y", ctypes.c_void_p)]


class Problem(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("in_", ctypes.c_int32), ("out", ctypes.c_int32),
                ("accumulate", ctypes.c_int32),
                ("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64),
                ("n", ctypes.c_int64), ("c", ctypes.c_int64), ("h", ctypes.c_int64),
                ("w", ctypes.c_int64), ("f", ctypes.c_int64), ("kh", ctypes.c_int64),
                ("kw", ctypes.c_int64),
                ("sh", ctypes.c_int32), ("sw", ctypes.c_int32), ("ph", ctypes.c_int32),
                ("pw", ctypes.c_int32),
                ("count", ctypes.c_int64), ("descs", ctypes.POINTER(GemmDesc))]


class TuneOpts(ctypes.Structure):
    _fields_ = [("strategy", ctypes.c_int32), ("budget_frac", ctypes.c_double),
                ("reps", ctypes.c_int32), ("warmup", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("db_path", ctypes.c_char_p), ("use_db", ctypes.c_int32),
                ("model", ctypes.c_void_p), ("times_us", ctypes.POINTER(ctypes.c_double)),
                ("fake_timer", ctypes.c_int32), ("table_us", ctypes.POINTER(ctypes.c_double))]


class TuneReport(ctypes.Structure):
    _fields_ = [("n_legal", ctypes.c_int32), ("n_measured", ctypes.c_int32),
                ("best_index", ctypes.c_int32), ("from_db", ctypes.c_int32),
                ("best_us", ctypes.c_double)]


_i32, _i64, _u32, _u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
_vp, _f, _int = ctypes.c_void_p, ctypes.c_float, ctypes.c_int
_st = ctypes.c_int
_cfgp = ctypes.POINTER(TileConfig)
_probp = ctypes.POINTER(Problem)

SIGNATURES = {
    "mlk_matmul": (_st, [_int, _int, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp,
                         _int, _cfgp, _vp]),
    "mlk_matmul_noalloc": (_st, [_int, _int, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp,
                                 _vp, _int, _cfgp, _vp]),
    "mlk_matmul_bias": (_st, [_int, _int, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _i64,
                              _vp, _vp, _int, _cfgp, _vp]),
    "mlk_conv2d_nchw_fchw": (_st, [_int, _int, _i64, _i64, _i64, _i64, _i64, _i64, _i64, _i32,
                                   _i32, _i32, _i32, _vp, _vp, _vp, _int, _cfgp, _vp]),
    "mlk_conv2d_plan_create": (_st, [_int, _int, _i64, _i64, _i64, _i64, _i64, _i64, _i64, _i32, _i32, _i32,
                                     _i32, _vp, _int, _cfgp, _vp, ctypes.POINTER(_vp)]),
    "mlk_conv2d_plan_run": (_st, [_vp, _vp, _vp, _vp]),
    "mlk_conv2d_plan_update_filter": (_st, [_vp, _vp]),
    "mlk_conv2d_plan_config": (_st, [_vp, _cfgp]),
    "mlk_conv2d_plan_destroy": (None, [_vp]),
    "mlk_conv2d_batch_create": (_st, [_int, _int, _i64, ctypes.POINTER(ConvDesc), _int, _cfgp, _vp,
                                      ctypes.POINTER(ctypes.c_void_p)]),
    "mlk_conv2d_batch_run": (_st, [_vp, _vp]),
    "mlk_conv2d_batch_update_filters": (_st, [_vp, _vp]),
    "mlk_conv2d_batch_info": (_st, [_vp, _cfgp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]),
    "mlk_conv2d_batch_destroy": (None, [_vp]),
    "mlk_mfma_rate": (_st, [_int, _i64, _vp, _i64, ctypes.POINTER(ctypes.c_int64), _vp]),
    "mlk_quantize": (_st, [_int, _i64, _vp, _vp, _vp, _vp]),
    "mlk_batched_matmul": (_st, [_int, _int, _i64, ctypes.POINTER(GemmDesc), _cfgp, _i64, _int, _u32,
                                 _vp]),
    "mlk_err_stats": (_st, [_int, _i64, _vp, _vp, _vp, _vp, _vp]),
    "mlk_tune": (_st, [_probp, ctypes.POINTER(TuneOpts), _cfgp, ctypes.POINTER(TuneReport)]),
    "mlk_config_legal": (_st, [_probp, _cfgp]),
    "mlk_config_count": (_i32, [_probp]),
    "mlk_config_get": (_st, [_probp, _i32, _cfgp]),
    "mlk_config_set_default": (_st, [_probp, _cfgp]),
    "mlk_model_feature_count": (_i32, []),
    "mlk_model_features": (_st, [_probp, _cfgp, ctypes.POINTER(_f)]),
    "mlk_model_create": (_st, [_i32, _u64, ctypes.POINTER(_vp)]),
    "mlk_model_destroy": (None, [_vp]),
    "mlk_model_add_sample": (_st, [_vp, _probp, _cfgp, ctypes.c_double]),
    "mlk_model_sample_count": (_i64, [_vp]),
    "mlk_model_train": (_st, [_vp, _i32, _i32, _f, ctypes.POINTER(_f)]),
    "mlk_model_predict": (_st, [_vp, _probp, _cfgp, _i32, ctypes.POINTER(_f)]),
    "mlk_mlp_forward": (_st, [_i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp]),
    "mlk_mlp_loss_grad": (_st, [_i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mlk_adam_step": (_st, [_i64, _vp, _vp, _vp, _vp, _f, _f, _f, _f, _i64, _vp]),
    "mlk_status_str": (ctypes.c_char_p, [_int]),
    "mlk_last_error": (ctypes.c_char_p, []),
    "mlk_version": (ctypes.c_char_p, []),
    "mlk_release": (None, []),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2307_16080_amd.build` "
                               "(or __graft_entry__.build()); there is no fallback path")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


class MlkError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")


def check(status):
    if status != MLK_OK:
        raise MlkError(status, lib().mlk_last_error().decode())
    return status
