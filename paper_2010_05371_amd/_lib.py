"""ctypes loader for libeapdtw.so (the C ABI declared in include/eapdtw.h)."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libeapdtw.so")

EAPDTW_OK = 0
EAPDTW_EINVAL = -1
EAPDTW_ENOMEM = -2
EAPDTW_EDEVICE = -3
EAPDTW_ENODEV = -4
EAPDTW_ENONFINITE = -5
EAPDTW_EPOISONED = -6

ERROR_NAMES = {
    EAPDTW_EINVAL: "EINVAL", EAPDTW_ENOMEM: "ENOMEM", EAPDTW_EDEVICE: "EDEVICE",
    EAPDTW_ENODEV: "ENODEV", EAPDTW_ENONFINITE: "ENONFINITE", EAPDTW_EPOISONED: "EPOISONED",
}


class Stats(ctypes.Structure):
    _fields_ = [("cells_nominal", ctypes.c_uint64), ("cells_evaluated", ctypes.c_uint64),
                ("cells_computed", ctypes.c_uint64), ("problems", ctypes.c_uint64),
                ("abandoned", ctypes.c_uint64), ("kernel_ms", ctypes.c_float),
                ("main_kernel_ms", ctypes.c_float)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class LbStats(ctypes.Structure):
    _fields_ = [("pruned_kim", ctypes.c_uint64), ("pruned_keogh_eq", ctypes.c_uint64),
                ("pruned_keogh_ec", ctypes.c_uint64), ("pruned_recheck", ctypes.c_uint64),
                ("dtw_candidates", ctypes.c_uint64),
                ("lb_ms", ctypes.c_float)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Query(ctypes.Structure):
    _fields_ = [("query", ctypes.c_void_p), ("m", ctypes.c_int64), ("window", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("dist", ctypes.c_double)]


class Pair(ctypes.Structure):
    """One pair of an uneven batch (eapdtw_pair)."""
    _fields_ = [("s_off", ctypes.c_int64), ("s_len", ctypes.c_int64), ("t_off", ctypes.c_int64),
                ("t_len", ctypes.c_int64), ("window", ctypes.c_int64)]


class Tune(ctypes.Structure):
    _fields_ = [("rows_per_group", ctypes.c_int64), ("border", ctypes.c_int64),
                ("check_interval", ctypes.c_int64), ("wide_rows", ctypes.c_int64),
                ("lanes", ctypes.c_int64), ("ms", ctypes.c_float)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load():
    """Loads the library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2010_05371_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, f32, f64 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_float,
                              ctypes.c_double)
    sp = ctypes.POINTER(Stats)
    lp = ctypes.POINTER(LbStats)
    sig = {
        "eapdtw_version": ([], ctypes.c_char_p),
        "eapdtw_create": ([i32, vp, ctypes.POINTER(vp)], i32),
        "eapdtw_destroy": ([vp], None),
        "eapdtw_set_stream": ([vp, vp], i32),
        "eapdtw_last_error": ([vp], ctypes.c_char_p),
        "eapdtw_set_option": ([vp, ctypes.c_char_p, i64], i32),
        "eapdtw_get_option": ([vp, ctypes.c_char_p, ctypes.POINTER(i64)], i32),
        "eapdtw_dtw": ([vp, vp, i64, vp, i64, i64, f64, ctypes.POINTER(f64), sp], i32),
        "eapdtw_dtw_pairs": ([vp, vp, vp, i64, i64, i64, i32, vp, vp, sp], i32),
        "eapdtw_pairwise": ([vp, vp, i64, i64, i64, vp, sp], i32),
        "eapdtw_nn_search": ([vp, vp, i64, vp, i64, i64, ctypes.POINTER(i64), ctypes.POINTER(f64),
                              sp], i32),
        "eapdtw_nn_search_noalloc": ([vp, vp, i64, vp, i64, i64, ctypes.POINTER(i64),
                                      ctypes.POINTER(f64)], i32),
        "eapdtw_nn_search_batch": ([vp, ctypes.POINTER(Query), i64, vp, i64,
                                    ctypes.POINTER(Result), sp], i32),
        "eapdtw_knn_search_batch": ([vp, ctypes.POINTER(Query), i64, vp, i64, i64,
                                     ctypes.POINTER(i64), ctypes.POINTER(f64), sp], i32),
        "eapdtw_dtw_ckpt_bytes": ([i64, i64, i64], i64),
        "eapdtw_dtw_fwd": ([vp, vp, vp, i64, i64, i64, vp, vp], i32),
        "eapdtw_dtw_bwd": ([vp, vp, vp, i64, i64, i64, vp, vp, vp, vp], i32),
        "eapdtw_dtw_path": ([vp, vp, vp, i64, i64, i64, vp, vp, vp], i32),
        "eapdtw_dtw_kernel_class": ([vp, i64, i64, i64, i32, ctypes.POINTER(i64),
                                     ctypes.POINTER(i64), ctypes.POINTER(i64)], i32),
        "eapdtw_dtw_pairs_batch": ([vp, vp, i64, vp, i64, ctypes.POINTER(Pair), i64, vp, vp, sp],
                                   i32),
        "eapdtw_dtw_batch_record_bytes": ([ctypes.POINTER(Pair), i64], i64),
        "eapdtw_dtw_batch_fwd": ([vp, vp, i64, vp, i64, ctypes.POINTER(Pair), i64, vp, vp], i32),
        "eapdtw_dtw_batch_bwd": ([vp, vp, i64, vp, i64, ctypes.POINTER(Pair), i64, vp, vp, vp, vp],
                                 i32),
        "eapdtw_dtw_batch_path": ([vp, vp, i64, vp, i64, ctypes.POINTER(Pair), i64, vp, vp], i32),
        "eapdtw_dba_step": ([vp, vp, i64, vp, i64, i64, i64, vp, vp], i32),
        "eapdtw_window_stats": ([vp, vp, i64, i64, vp, vp], i32),
        "eapdtw_znorm": ([vp, vp, i64, vp], i32),
        "eapdtw_nn_dists": ([vp, vp, i64, vp, i64, i64, f32, vp, sp], i32),
        "eapdtw_autotune": ([vp, vp, i64, vp, i64, i64, i64, ctypes.POINTER(Tune)], i32),
        "eapdtw_tune_bucket": ([i64, i64], i64),
        "eapdtw_tune_get": ([vp, i64, ctypes.POINTER(Tune)], i32),
        "eapdtw_tune_save": ([vp, ctypes.c_char_p], i32),
        "eapdtw_tune_load": ([vp, ctypes.c_char_p], i32),
        "eapdtw_nn_search_lb": ([vp, vp, i64, vp, i64, i64, ctypes.POINTER(i64),
                                 ctypes.POINTER(f64), sp, lp], i32),
        "eapdtw_nn_dists_lb": ([vp, vp, i64, vp, i64, i64, f32, vp, sp, lp], i32),
        "eapdtw_nn_lower_bounds": ([vp, vp, i64, vp, i64, i64, vp, vp, vp], i32),
        "eapdtw_knn_search": ([vp, vp, i64, vp, i64, i64, i64, ctypes.POINTER(i64),
                               ctypes.POINTER(f64), sp], i32),
        "eapdtw_erp_pairs": ([vp, vp, vp, i64, i64, i64, f64, vp, vp, sp], i32),
        "eapdtw_nn_search_erp": ([vp, vp, i64, vp, i64, i64, f64, ctypes.POINTER(i64),
                                  ctypes.POINTER(f64), sp], i32),
        "eapdtw_knn_search_lb": ([vp, vp, i64, vp, i64, i64, i64, ctypes.POINTER(i64),
                                  ctypes.POINTER(f64), sp, lp], i32),
        "eapdtw_nn1": ([vp, vp, i64, i64, i64, ctypes.POINTER(i64), ctypes.POINTER(f64), sp], i32),
        "eapdtw_nn1_ref": ([vp, vp, i64, vp, i64, i64, i64, ctypes.POINTER(i64), ctypes.POINTER(f64),
                            sp], i32),
        "eapdtw_nn_search_w": ([vp, vp, i64, vp, i64, i64, f32, ctypes.POINTER(i64),
                                ctypes.POINTER(f64), sp], i32),
        "eapdtw_nn_dists_w": ([vp, vp, i64, vp, i64, i64, f32, f32, vp, sp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class EapdtwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code
