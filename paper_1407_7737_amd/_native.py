"""ctypes binding of libcurob.so (include/curob.h), argument marshalling only.

Device buffers are torch tensors on the GPU (or raw integer device addresses); every
evaluation runs in the library's HIP kernels.  There is no CPU fallback: importing this
module without the built library raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcurob.so")

CUROB_OK = 0
CUROB_E_STATE = -1
CUROB_E_ARG = -2
CUROB_E_FID = -3
CUROB_E_CAPACITY = -4
CUROB_E_HIP = -5
MODE_SPLIT = 0
MODE_FP32 = 1
MODE_SPLIT_BF16X3 = 2
MODE_SPLIT_BF16X6 = 3
CUSTOM_ID_MIN = 64
CUSTOM_ID_MAX = 1023
NOALLOC_SCRATCH_BYTES = 32 << 20

EXPORTED = [
    "initialize", "dispose", "func_evaluate", "func_evaluatef", "h_func_evaluate", "h_func_evaluatef",
    "curob_set_stream", "curob_set_mode", "curob_define_basic", "curob_define_hybrid",
    "curob_define_composition", "curob_last_error", "curob_get_problem", "curob_generate_basic",
    "curob_batch_create", "curob_batch_bind", "curob_batch_run", "curob_batch_run_direct",
    "curob_batch_configure", "curob_batch_shape", "curob_batch_tune", "curob_batch_destroy",
    "curob_probe_read", "curob_probe_mfma_bf16", "curob_get_dim", "curob_get_info", "curob_get_structure",
    "curob_get_composition", "curob_generate_info", "curob_generate_structure", "curob_generate_composition",
    "func_evaluatef_noalloc", "curob_de_run", "curob_shape_key", "curob_set_shape", "curob_tune",
]
BATCH_KEY_BASE = 2048  # population i of a batch keys its random data like custom id 2048 + i


class CurobError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"curob error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python paper_1407_7737_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    i32, u64, vp = ctypes.c_int, ctypes.c_ulonglong, ctypes.c_void_p
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    sig = {
        "initialize": (i32, [i32, i32, u64]),
        "dispose": (i32, []),
        "func_evaluate": (i32, [i32, vp, i32, vp]),
        "func_evaluatef": (i32, [i32, vp, i32, vp]),
        "func_evaluatef_noalloc": (i32, [i32, vp, i32, vp]),
        "curob_shape_key": (i32, [i32, i32, i32, ip]),
        "curob_set_shape": (i32, [ip, i32, i32]),
        "curob_tune": (i32, [i32, i32, vp, i32, vp, i32, ip, ip, ctypes.POINTER(ctypes.c_float),
                             ctypes.POINTER(ctypes.c_float), i32, ip]),
        "curob_de_run": (i32, [i32, i32, i32, ctypes.c_double, ctypes.c_double, u64, vp, vp, vp, vp, vp, i32]),
        "h_func_evaluate": (i32, [i32, vp, i32, vp]),
        "h_func_evaluatef": (i32, [i32, vp, i32, vp]),
        "curob_set_stream": (i32, [vp]),
        "curob_set_mode": (i32, [i32]),
        "curob_define_basic": (i32, [i32, i32, ctypes.c_double, ctypes.c_double, i32]),
        "curob_define_hybrid": (i32, [i32, i32, ip, dp]),
        "curob_define_composition": (i32, [i32, i32, ip, dp, dp, dp]),
        "curob_last_error": (ctypes.c_char_p, []),
        "curob_get_problem": (i32, [i32, dp, dp]),
        "curob_generate_basic": (i32, [i32, i32, u64, dp, dp]),
        "curob_batch_create": (i32, [i32, ip, ip, ip, u64, ctypes.POINTER(vp)]),
        "curob_batch_bind": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
        "curob_batch_run": (i32, [vp]),
        "curob_batch_run_direct": (i32, [vp]),
        "curob_batch_configure": (i32, [vp, i32, i32, i32]),
        "curob_batch_shape": (i32, [vp, ip, ip, ip, ip]),
        "curob_batch_tune": (i32, [vp, i32, ctypes.POINTER(ctypes.c_float)]),
        "curob_batch_destroy": (i32, [vp]),
        "curob_probe_read": (i32, [vp, u64, i32, ctypes.POINTER(ctypes.c_double)]),
        "curob_probe_mfma_bf16": (i32, [i32, ctypes.POINTER(ctypes.c_double)]),
        "curob_get_dim": (i32, [ip, ip]),
        "curob_get_info": (i32, [i32, i32, ip, ip, ip]),
        "curob_get_structure": (i32, [i32, i32, dp, ip, ip, dp, ip, dp, dp]),
        "curob_get_composition": (i32, [i32, dp, dp, dp]),
        "curob_generate_info": (i32, [i32, i32, u64, i32, ip, ip, ip]),
        "curob_generate_structure": (i32, [i32, i32, u64, i32, dp, ip, ip, dp, ip, dp, dp]),
        "curob_generate_composition": (i32, [i32, i32, u64, dp, dp, dp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


def last_error() -> str:
    return (lib.curob_last_error() or b"").decode()


def check(rc: int) -> int:
    if rc != CUROB_OK:
        raise CurobError(rc, last_error())
    return rc
