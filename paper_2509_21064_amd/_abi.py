"""ctypes mirror of include/pdbo.h and the loader of libpdbo.so.

Argument marshalling only: every step of the method runs in the HIP library.
There is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_uint8, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpdbo.so")

PDBO_OK, PDBO_EINVAL, PDBO_ENOMEM, PDBO_EDEVICE, PDBO_ERANGE, PDBO_ESTATE, PDBO_EUNSUPPORTED = range(7)
PDBO_DENSE, PDBO_CSR = 0, 1
PDBO_G_QUAD, PDBO_G_ENTROPY, PDBO_G_POLY = 0, 1, 2
PDBO_DUAL_VECTOR, PDBO_DUAL_SCALAR = 0, 1
PDBO_FP32, PDBO_BF16, PDBO_FP8, PDBO_I8 = 0, 1, 2, 3
PDBO_W_INT32, PDBO_W_F64 = 0, 1
PDBO_K_STEP, PDBO_K_EVAL, PDBO_K_ARGMIN, PDBO_K_PERSISTENT, PDBO_K_INCR = 0, 1, 2, 3, 4


class pdbo_qubo(ctypes.Structure):
    _fields_ = [("n", c_int32), ("format", c_int32), ("q", c_void_p), ("row_ptr", c_void_p),
                ("col_idx", c_void_p), ("nnz", c_int64), ("c", c_void_p), ("wtype", c_int32),
                ("_pad", c_int32), ("qd", c_void_p), ("cd", c_void_p)]


class pdbo_maxsat(ctypes.Structure):
    _fields_ = [("n", c_int32), ("m", c_int32), ("k", c_int32), ("lits", c_void_p), ("w", c_void_p)]


class pdbo_kcut(ctypes.Structure):
    _fields_ = [("n", c_int32), ("k", c_int32), ("row_ptr", c_void_p), ("col_idx", c_void_p),
                ("w", c_void_p), ("nnz", c_int64)]


class pdbo_params(ctypes.Structure):
    _fields_ = [("B", c_int32), ("g_kind", c_int32), ("precision", c_int32), ("eval_every", c_int32),
                ("alpha", c_double), ("beta", c_double), ("y0", c_double), ("delta", c_double),
                ("scale", c_double), ("tile", c_int32), ("graph_chunk", c_int32),
                ("g_degree", c_int32), ("dual_kind", c_int32), ("x0", c_void_p), ("seed", c_uint64)]


class pdbo_result(ctypes.Structure):
    _fields_ = [("best_obj", c_int64), ("best_restart", c_int32), ("_pad", c_int32),
                ("best_iter", c_int64), ("time_to_best_s", c_double), ("steps_done", c_int64),
                ("best_x", c_void_p), ("best_obj_f64", c_double)]


_ctx = c_void_p
_st = c_int32

# name -> (restype, argtypes); exactly the entry points declared in include/pdbo.h
SIGNATURES = {
    "qubo_gda_init": (_st, [POINTER(pdbo_qubo), POINTER(pdbo_params), c_void_p, POINTER(_ctx)]),
    "qubo_gda_step": (_st, [_ctx, c_int32]),
    "qubo_gda_result": (_st, [_ctx, POINTER(pdbo_result)]),
    "qubo_gda_get_state": (_st, [_ctx, c_void_p, c_void_p, POINTER(c_int64)]),
    "qubo_gda_set_state": (_st, [_ctx, c_void_p, c_void_p, c_int64]),
    "qubo_gda_restart": (_st, [_ctx, c_void_p]),
    "qubo_gda_objectives": (_st, [_ctx, c_void_p]),
    "qubo_gda_objectives_f64": (_st, [_ctx, c_void_p]),
    "qubo_gda_grad": (_st, [_ctx, c_void_p, c_void_p]),
    "qubo_gda_eval": (_st, [_ctx, c_void_p, c_int32, c_void_p]),
    "qubo_gda_eval_f64": (_st, [_ctx, c_void_p, c_int32, c_void_p]),
    "qubo_gda_eval_noalloc": (_st, [_ctx, c_void_p, c_int32, c_void_p, c_void_p]),
    "qubo_dual_bound": (_st, [_ctx, c_double, c_int32, POINTER(c_double), c_void_p, c_void_p]),
    "qubo_gda_solve": (_st, [POINTER(pdbo_qubo), POINTER(pdbo_params), c_int32, c_void_p,
                             POINTER(pdbo_result)]),
    "qubo_gda_batch_init": (_st, [c_int32, POINTER(pdbo_qubo), POINTER(pdbo_params), c_int32,
                                  c_void_p, POINTER(_ctx)]),
    "qubo_gda_batch_result": (_st, [_ctx, c_int32, POINTER(pdbo_result)]),
    "qubo_gda_batch_solve": (_st, [c_int32, POINTER(pdbo_qubo), POINTER(pdbo_params), c_int32,
                                   c_int32, c_void_p, POINTER(pdbo_result)]),
    "kcut_gda_init": (_st, [POINTER(pdbo_kcut), POINTER(pdbo_params), c_void_p, POINTER(_ctx)]),
    "maxsat_gda_init": (_st, [POINTER(pdbo_maxsat), POINTER(pdbo_params), c_void_p, POINTER(_ctx)]),
    "maxsat_gda_step": (_st, [_ctx, c_int32]),
    "maxsat_gda_result": (_st, [_ctx, POINTER(pdbo_result)]),
    "maxsat_gda_solve": (_st, [POINTER(pdbo_maxsat), POINTER(pdbo_params), c_int32, c_void_p,
                               POINTER(pdbo_result)]),
    "maxsat_lagrangian_fwd": (_st, [_ctx, c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "maxsat_lagrangian_bwd": (_st, [_ctx, c_void_p, c_void_p, c_void_p, c_int32, c_void_p,
                                    c_void_p, c_void_p]),
    "qubo_gda_trace": (_st, [_ctx, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                             POINTER(c_int32)]),
    "qubo_gda_trace_f64": (_st, [_ctx, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                 POINTER(c_int32)]),
    "pdbo_timing": (_st, [_ctx, c_int32]),
    "pdbo_timing_classes": (_st, [_ctx, c_uint32]),
    "pdbo_timing_stride": (_st, [_ctx, c_int32]),
    "pdbo_kernel_time": (_st, [_ctx, c_int32, POINTER(c_double), POINTER(c_int64)]),
    "pdbo_tile_name": (c_char_p, [_ctx]),
    "pdbo_autotune_store": (_st, [c_char_p, c_int32]),
    "pdbo_autotune_lookup": (_st, [c_char_p, POINTER(c_int32)]),
    "pdbo_destroy": (None, [_ctx]),
    "pdbo_status_str": (c_char_p, [c_int32]),
    "pdbo_last_error": (c_char_p, [_ctx]),
    "pdbo_last_global_error": (c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libpdbo.so once; raises RuntimeError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpdbo.so not found at {path}: build it with "
                           "`python -m paper_2509_21064_amd.build` (there is no fallback path)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class PdboError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = status
        super().__init__(f"[{status}] {msg}")


def check(status: int, ctx=None):
    if status != PDBO_OK:
        lib = load()
        what = lib.pdbo_status_str(status).decode()
        detail = (lib.pdbo_last_error(ctx) if ctx else lib.pdbo_last_global_error()).decode()
        raise PdboError(status, f"{what}: {detail}")
