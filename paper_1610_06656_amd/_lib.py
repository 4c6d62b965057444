"""ctypes declarations of the C-ABI in include/smp.h.

Loading fails loudly (RuntimeError) when libsmp.so is missing: there is no CPU
fallback for any entry point.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmp.so")

SMP_OK = 0
SMP_ERR_INVALID_ARG = 1
SMP_ERR_OUT_OF_MEMORY = 2
SMP_ERR_DEVICE = 3
SMP_ERR_NUMERIC = 4
SMP_ERR_CAPACITY = 5
SMP_ERR_STATE = 6
SMP_ERR_BUSY = 7

SMP_PREC_FP32 = 0
SMP_PREC_BF16 = 1
SMP_PREC_FP8 = 2
SMP_OMEGA_REUSE = 0
SMP_OMEGA_SPLIT = 1
SMP_B_IS_A = 1
SMP_SAMPLE_MULTINOMIAL = 2
SMP_SKETCH_SRHT = 4
SMP_MAT_A = 0
SMP_MAT_B = 1


class SmpParams(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int64), ("n1", ctypes.c_int64), ("n2", ctypes.c_int64),
        ("k", ctypes.c_int32), ("r", ctypes.c_int32), ("T", ctypes.c_int32),
        ("prec", ctypes.c_int32), ("omega_mode", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("m", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("init_iters", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class SmpOmega(ctypes.Structure):
    _fields_ = [
        ("n1", ctypes.c_int64), ("n2", ctypes.c_int64), ("cap", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("w_csr", ctypes.c_void_p),
        ("mt_csr", ctypes.c_void_p), ("sub_csr", ctypes.c_void_p),
        ("col_ptr", ctypes.c_void_p), ("row_idx", ctypes.c_void_p), ("w_csc", ctypes.c_void_p),
        ("mt_csc", ctypes.c_void_p), ("sub_csc", ctypes.c_void_p),
    ]


class SmpJobResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("worker", ctypes.c_int32),
                ("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double)]


class SmpServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("max_running", ctypes.c_int32), ("workers", ctypes.c_int32),
                ("max_budget_in_use", ctypes.c_int64), ("refused", ctypes.c_int64)]


EXPORTS = {
    # name: (restype, argtypes)
    "smp_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_void_p]),
    "smp_destroy": (None, [ctypes.c_void_p]),
    "smp_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "smp_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "smp_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "smp_check_params": (ctypes.c_int, [ctypes.POINTER(SmpParams)]),
    "smp_workspace_size": (ctypes.c_int, [ctypes.POINTER(SmpParams), ctypes.POINTER(ctypes.c_size_t)]),
    "smp_pi_fill": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_void_p]),
    "smp_sketch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "smp_sketch_begin": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.POINTER(ctypes.c_void_p)]),
    "smp_sketch_push": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]),
    "smp_sketch_end": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "smp_sketch_free": (None, [ctypes.c_void_p]),
    "smp_sketch_push_coo": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]),
    "smp_sketch_push_csr": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int64]),
    "smp_sketch_group": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(SmpParams),
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                        ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p)]),
    "smp_waltmin_group": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(SmpParams),
                                         ctypes.POINTER(SmpOmega), ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]),
    "smp_tune_sketch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "smp_tune_lookup": (ctypes.c_int, [ctypes.POINTER(SmpParams), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "smp_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "smp_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "smp_tune_clear": (None, []),
    "smp_solve_sketched": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "smp_sample": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.POINTER(SmpOmega)]),
    "smp_estimate": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(SmpOmega)]),
    "smp_svd_sketch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "smp_solve_svd_sketch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_void_p,
                                            ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "smp_column_norms": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "smp_exact_entries": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.POINTER(SmpOmega)]),
    "smp_lela": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_void_p, ctypes.c_int64,
                                ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "smp_estimate_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(SmpOmega)]),
    "smp_waltmin": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.POINTER(SmpOmega),
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "smp_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "smp_stage_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float), ctypes.c_int]),
    "smp_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_void_p, ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p]),
    "smp_server_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_size_t,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "smp_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "smp_server_try_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpParams), ctypes.c_void_p,
                                             ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "smp_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(SmpJobResult)]),
    "smp_server_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "smp_server_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SmpServerStats)]),
    "smp_server_destroy": (None, [ctypes.c_void_p]),
    "smp_solve_batch_group": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(SmpParams),
                                             ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                             ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int,
                                             ctypes.POINTER(SmpJobResult)]),
    "smp_solve_batch": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(SmpParams),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_size_t,
                                       ctypes.POINTER(SmpJobResult)]),
}

_lib = None


def load():
    """Load libsmp.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1610_06656_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
