"""ctypes view of libspgemm.so (the C ABI declared in include/spgemm.h).

Loading fails loudly when the library has not been built: there is no CPU
fallback for any entry point.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspgemm.so")

OK = 0
EINVAL = -1
ENOMEM = -2
EHIP = -3
EUNSUPPORTED = -4
ESTATE = -5

F32 = 0
F64 = 1

_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHIP: "EHIP",
          EUNSUPPORTED: "EUNSUPPORTED", ESTATE: "ESTATE"}


class SpgemmError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {_NAMES.get(code, code)}: {msg}")
        self.code = code


class Csc(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("colptr", ctypes.c_void_p), ("rowidx", ctypes.c_void_p),
                ("vals", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("tiny_max_flop", ctypes.c_int32), ("hash_max_flop", ctypes.c_int32),
                ("hash_max_nnz", ctypes.c_int32), ("dense_window", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("own_partition", ctypes.c_int32),
                ("own_partition_whole", ctypes.c_int32), ("medium_kernel", ctypes.c_int32),
                ("batch_streams", ctypes.c_int32), ("batch_form", ctypes.c_int32),
                ("dense_first_flop", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("workspace_limit", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("k", ctypes.c_int64), ("n", ctypes.c_int64),
                ("nnz_A", ctypes.c_int64), ("nnz_B", ctypes.c_int64),
                ("h_count", ctypes.c_int64), ("nzc_A", ctypes.c_int64), ("K", ctypes.c_int64),
                ("M", ctypes.c_int64), ("kt", ctypes.c_int64), ("nnz_At", ctypes.c_int64),
                ("cv_memA", ctypes.c_double), ("flops", ctypes.c_int64),
                ("nnz_C", ctypes.c_int64), ("sym_bins", ctypes.c_int64 * 8),
                ("num_bins", ctypes.c_int64 * 8)]


class BatchIO(ctypes.Structure):
    _fields_ = [("A_vals", ctypes.c_void_p), ("B_vals", ctypes.c_void_p),
                ("C_rowidx", ctypes.c_void_p), ("C_vals", ctypes.c_void_p),
                ("dep_A", ctypes.c_int32), ("dep_B", ctypes.c_int32)]


# every symbol include/spgemm.h declares, with its ctypes signature
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
SIGNATURES = {
    "spgemm_last_error": (ctypes.c_char_p, []),
    "spgemm_version": (ctypes.c_char_p, []),
    "spgemm_default_tuning": (ctypes.c_int, [ctypes.POINTER(Tuning)]),
    "spgemm_plan": (ctypes.c_int, [ctypes.POINTER(Csc), ctypes.POINTER(Csc), ctypes.c_int,
                                   _vp, _i32, _i64,
                                   ctypes.POINTER(Tuning), _vp, ctypes.POINTER(_vp)]),
    "spgemm_plan_set_stream": (ctypes.c_int, [_vp, _vp]),
    "spgemm_plan_stats": (ctypes.c_int, [_vp, ctypes.POINTER(Stats)]),
    "spgemm_plan_export": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "spgemm_plan_export_bins": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "spgemm_symbolic": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_int64)]),
    "spgemm_symbolic_noalloc": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_int64)]),
    "spgemm_numeric": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "spgemm_backward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "spgemm_plan_destroy": (ctypes.c_int, [_vp]),
    "spgemm_batch_create": (ctypes.c_int, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(BatchIO),
                                           ctypes.POINTER(Tuning), ctypes.POINTER(_vp)]),
    "spgemm_batch_run": (ctypes.c_int, [_vp, _i32, _vp]),
    "spgemm_batched": (ctypes.c_int, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(BatchIO), _i32,
                                      _vp]),
    "spgemm_batch_info": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "spgemm_batch_check": (ctypes.c_int, [_vp]),
    "spgemm_batch_destroy": (ctypes.c_int, [_vp]),
    "spgemm_row_block": (ctypes.c_int, [ctypes.POINTER(Csc), ctypes.c_int, _i64, _i64, _vp, _vp,
                                        _vp, _vp]),
    "spgemm_stack_parts": (ctypes.c_int, [_i32, ctypes.POINTER(Csc), ctypes.c_int, _vp, _vp, _vp,
                                          _vp, _vp, _vp, _vp]),
    "spgemm_pool_trim": (ctypes.c_int, []),
}

_lib = None


def load(path: str = None):
    """Loads the in-tree libspgemm.so once and returns it; raises if it is
    missing.  `path` names another build of the same sources (for example one
    compiled with different settings by build.build(out=...)); it is honoured
    only by the first call of the process, and the product never passes it."""
    global _lib
    if _lib is not None:
        if path is not None and getattr(_lib, "_name", None) != path:
            raise RuntimeError(f"{_lib._name} is already loaded")
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: the HIP library is required "
                           "(build it with __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int, where: str):
    if code != OK:
        msg = load().spgemm_last_error().decode(errors="replace")
        raise SpgemmError(code, where, msg)
