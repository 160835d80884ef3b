"""ctypes loader for libbfgpa.so (the C ABI declared in include/bf_gpa.h).

The library is built in-tree by ``paper_1603_08109_amd.build``.  There is no
fallback: if the shared object is missing or does not load, every entry point
raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libbfgpa.so")

BF_OK = 0
BF_EINVAL = -1
BF_ENOMEM = -2
BF_EHIP = -3
BF_EUNSUPPORTED = -4
BF_WNOGUARANTEE = 1

BF_BOX = 0
BF_GAUSS = 1
BF_GAUSS_REC = 2

BF_NRULE_LAMBERTW = 0
BF_NRULE_ALG1 = 1
BF_NRULE_POISSON = 2

BF_FLAG_FP32_ACCUM = 1
BF_FLAG_GRAD = 2
BF_FLAG_STREAMED = 4
BF_FLAG_JOINT = 8
BF_FLAG_MIRROR = 16
BF_FLAG_TILE_VALU = 32
BF_FLAG_MFMA_FP32 = 128
BF_PATH_TILE = 0
BF_PATH_STREAMED = 1
BF_PATH_RECURSIVE = 3
BF_PATH_VOLUME = 4
BF_PATH_WIDE = 5


class bf_params(C.Structure):
    _fields_ = [
        ("kernel", C.c_int32),
        ("sigma_s", C.c_double),
        ("W", C.c_int32),
        ("sigma_r", C.c_double),
        ("T", C.c_double),
        ("center", C.c_double),
        ("N", C.c_int32),
        ("delta", C.c_double),
        ("n_rule", C.c_int32),
        ("height", C.c_int32),
        ("width", C.c_int32),
        ("flags", C.c_int32),
    ]


class bf_batch_info(C.Structure):
    _fields_ = [
        ("images_persistent", C.c_int32),
        ("images_streamed", C.c_int32),
        ("persistent_lds_bytes", C.c_int64),
        ("workspace_bytes", C.c_int64),
        ("forward_graph_launches", C.c_int64),
        ("forward_direct_launches", C.c_int64),
        ("backward_graph_launches", C.c_int64),
        ("backward_direct_launches", C.c_int64),
    ]


class bf_plan_info(C.Structure):
    _fields_ = [
        ("N", C.c_int32),
        ("W", C.c_int32),
        ("w0", C.c_double),
        ("eps", C.c_double),
        ("lambda_", C.c_double),
        ("kernel_bound", C.c_double),
        ("guaranteed_delta", C.c_double),
        ("tile_rows", C.c_int32),
        ("tile_cols", C.c_int32),
        ("workspace_bytes", C.c_int64),
        ("path", C.c_int32),
    ]


# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "bf_order": (C.c_int, [C.POINTER(bf_params), C.POINTER(bf_plan_info)]),
    "bf_plan": (C.c_int, [C.POINTER(bf_params), C.POINTER(C.c_void_p)]),
    "bf_plan_get_info": (C.c_int, [C.c_void_p, C.POINTER(bf_plan_info)]),
    "bf_destroy": (C.c_int, [C.c_void_p]),
    "bf_plan_clone_workspace": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "bf_plan_volume": (C.c_int, [C.POINTER(bf_params), C.c_int32, C.POINTER(C.c_void_p)]),
    "bf_forward_volume": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    "bf_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                             C.c_void_p]),
    "bf_forward_noalloc": (C.c_int, [C.POINTER(bf_params), C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                     C.c_void_p]),
    "bf_forward_joint": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                   C.c_int64, C.c_void_p]),
    "bf_image_range": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "bf_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                              C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "bf_batch_plan": (C.c_int, [C.c_int32, C.POINTER(bf_params), C.POINTER(C.c_void_p)]),
    "bf_batch_forward": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.c_void_p]),
    "bf_batch_status": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "bf_batch_get_info": (C.c_int, [C.c_void_p, C.POINTER(bf_batch_info)]),
    "bf_batch_tune": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.c_void_p,
                                C.POINTER(C.c_int32)]),
    "bf_batch_backward": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.POINTER(C.c_void_p),
                                    C.POINTER(C.c_int64), C.c_void_p, C.c_void_p]),
    "bf_batch_forward_saved": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.POINTER(C.c_void_p),
                                         C.c_void_p]),
    "bf_batch_backward_saved": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                          C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.POINTER(C.c_void_p),
                                          C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.c_void_p, C.c_void_p]),
    "bf_batch_destroy": (C.c_int, [C.c_void_p]),
    "bf_status_string": (C.c_char_p, [C.c_int]),
    "bf_last_error_message": (C.c_char_p, []),
    "bf_version": (C.c_char_p, []),
}

_lock = threading.Lock()
_lib = None


def load() -> C.CDLL:
    """Load libbfgpa.so (once).  Raises RuntimeError if it is not built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1603_08109_amd.build` "
                "(there is no CPU fallback)")
        lib = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


class BFError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = load()
        msg = lib.bf_last_error_message().decode(errors="replace")
        super().__init__(f"{where}: {lib.bf_status_string(code).decode()} ({code}): {msg}")
        self.code = code


def check(code: int, where: str) -> int:
    if code < 0:
        raise BFError(code, where)
    return code
