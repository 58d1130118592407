"""ctypes binding of libhdconv.so (the C ABI in include/hdconv.h).

Argument marshalling only: every step of a convolution runs in the library's
HIP kernels.  PyTorch provides device memory and the stream.  If the library
is missing this module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhdconv.so")

C64, C128 = 0, 1
OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, ENODEV = 0, -1, -2, -3, -4, -5
METHOD_AUTO, METHOD_HYBRID, METHOD_EXPLICIT = 0, 1, 2
VARIANT_AUTO, VARIANT_FUSED, VARIANT_MULTIPASS, VARIANT_OUTER = 0, 1, 2, 3
PLAN_HOST_ONLY = 1
BATCH_NO_GRAPH = 2
PLAN_CENTERED = 4
PLAN_HERMITIAN = 8
PLAN_NO_WORKSPACE = 16
PLAN_ACCUMULATE_OUTPUT = 32
BATCH_GROUPED = 64
SCRATCH_BYTES = 64 << 20  # static scratch of hdconv_execute_noalloc
MULT_PRODUCT, MULT_QUADRATIC = 0, 1
TUNER_HEURISTIC, TUNER_EXHAUSTIVE, TUNER_MODEL = 0, 1, 2
NFEATURES = 48

VARIANT_NAMES = {0: "auto", 1: "fused", 2: "multipass", 3: "outer"}
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSUPPORTED", -5: "ENODEV"}

_i64 = ctypes.c_int64


class Options(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("flags", ctypes.c_int),
                ("m", _i64 * 3), ("p", _i64 * 3), ("D", _i64 * 3),
                ("variant", ctypes.c_int * 3), ("E_m", ctypes.c_int * 3), ("E_p", ctypes.c_int * 3),
                ("S", ctypes.c_int * 3), ("rows_per_block", ctypes.c_int * 3), ("twiddles", ctypes.c_int * 3),
                ("tuner", ctypes.c_int), ("tune_reps", ctypes.c_int), ("margin", ctypes.c_double),
                ("model", ctypes.c_void_p), ("db_path", ctypes.c_char_p), ("copies", _i64), ("dist", _i64),
                ("mult", ctypes.c_int), ("mult_coef", ctypes.POINTER(ctypes.c_double)), ("stride", _i64 * 2),
                ("conj_pairs", ctypes.c_int), ("reserved", ctypes.c_int * 7)]


class DimInfo(ctypes.Structure):
    _fields_ = [("L", _i64), ("M", _i64), ("m", _i64), ("p", _i64), ("n", _i64), ("q", _i64),
                ("D", _i64), ("variant", ctypes.c_int), ("E_m", ctypes.c_int), ("E_p", ctypes.c_int),
                ("S", ctypes.c_int), ("rows_per_block", ctypes.c_int), ("tw_m", ctypes.c_int),
                ("tw_p", ctypes.c_int), ("centered", ctypes.c_int)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int), ("A", ctypes.c_int), ("B", ctypes.c_int), ("dtype", ctypes.c_int),
                ("method", ctypes.c_int), ("L", _i64 * 3), ("M", _i64 * 3), ("dim", DimInfo * 3),
                ("npad", _i64 * 3), ("workspace_bytes", ctypes.c_size_t), ("table_bytes", ctypes.c_size_t),
                ("compulsory_bytes", ctypes.c_double), ("traffic_bytes", ctypes.c_double),
                ("launches", ctypes.c_int), ("tuner", ctypes.c_int), ("tuned_candidates", ctypes.c_int),
                ("timed_candidates", ctypes.c_int), ("tuned_ms", ctypes.c_double)]


class BatchStats(ctypes.Structure):
    _fields_ = [("persistent", ctypes.c_int), ("grid", ctypes.c_int), ("tasks", _i64), ("lds_bytes", _i64),
                ("work_bytes", _i64)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", _i64), ("total_ms", ctypes.c_double),
                ("bytes_per_launch", ctypes.c_double)]


# every symbol include/hdconv.h declares, with its signature
SIGNATURES = {
    "hdconv_options_init": (None, [ctypes.POINTER(Options)]),
    "hdconv_plan": (ctypes.c_void_p, [ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_int]),
    "hdconv_plan_ex": (ctypes.c_void_p, [ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.POINTER(Options)]),
    "hdconv_execute": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "hdconv_execute_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                              ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "hdconv_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(PlanInfo)]),
    "hdconv_destroy": (None, [ctypes.c_void_p]),
    "hdconv_geometry": (ctypes.c_int, [_i64, _i64, _i64, _i64, ctypes.c_int, ctypes.POINTER(DimInfo)]),
    "hdconv_geometry_ex": (ctypes.c_int, [_i64, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(DimInfo)]),
    "hdconv_centered_span": (_i64, [_i64, _i64]),
    "hdconv_min_padding": (ctypes.c_int, [_i64, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_i64)]),
    "hdconv_candidates": (ctypes.c_int, [ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(DimInfo),
                                         ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "hdconv_time_shape": (ctypes.c_int, [ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.POINTER(DimInfo), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_double)]),
    "hdconv_features": (ctypes.c_int, [ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.POINTER(DimInfo),
                                       ctypes.POINTER(ctypes.c_float)]),
    "hdconv_model_create": (ctypes.c_void_p, [ctypes.c_int, ctypes.c_uint64]),
    "hdconv_model_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_int)]),
    "hdconv_model_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_int]),
    "hdconv_model_train": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                          ctypes.POINTER(ctypes.c_float), _i64, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_float, ctypes.c_uint64, ctypes.POINTER(ctypes.c_float)]),
    "hdconv_model_predict": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), _i64,
                                            ctypes.POINTER(ctypes.c_float)]),
    "hdconv_model_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                         ctypes.POINTER(ctypes.c_float), _i64, ctypes.POINTER(ctypes.c_float),
                                         ctypes.POINTER(ctypes.c_float)]),
    "hdconv_model_destroy": (None, [ctypes.c_void_p]),
    "hdconv_plan_batched": (ctypes.c_void_p, [ctypes.POINTER(_i64), ctypes.POINTER(_i64), _i64, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Options)]),
    "hdconv_execute_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                              ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]),
    "hdconv_batch_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(DimInfo), ctypes.POINTER(_i64),
                                         ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "hdconv_batch_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(BatchStats)]),
    "hdconv_batch_destroy": (None, [ctypes.c_void_p]),
    "hdconv_profile_begin": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "hdconv_profile_end": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(KernelStat), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int)]),
    "hdconv_last_error": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_size_t]),
    "hdconv_version": (ctypes.c_char_p, []),
}

_lock = threading.Lock()
_lib = None


class HdconvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, str(code)), msg))
        self.code = code


def _bind_runtime_first():
    """Load PyTorch (when installed) before the library.  PyTorch ships its
    own HIP runtime under the same soname as the system's; whichever is
    loaded first serves the process.  Loaded first, the library binds to the
    system runtime, PyTorch then finds no device, and the library's kernels
    measured up to 30 % slower (256^3 plan 1.50 against 1.13 ms), so the
    front end, whose tensors are PyTorch's, always loads PyTorch first."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("libhdconv.so is not built (run python -m paper_2303_17510_amd.build): %s"
                                  % LIB_PATH)
            _bind_runtime_first()
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def last_error():
    buf = ctypes.create_string_buffer(512)
    code = lib().hdconv_last_error(buf, 512)
    return code, buf.value.decode(errors="replace")


def check(rc: int):
    if rc != OK:
        code, msg = last_error()
        raise HdconvError(rc, msg)
