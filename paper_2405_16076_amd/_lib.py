"""ctypes declarations of include/rid.h (argument marshalling only).

Loading fails loudly when librid.so has not been built: there is no CPU
fallback for any entry point.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librid.so")

RID_OK, RID_EINVAL, RID_ENOMEM, RID_EDEVICE, RID_ESTATE, RID_ECAPACITY, RID_ENUMERIC, RID_ENOTSUP = range(8)
RID_F32, RID_F64 = 0, 1
RID_SKETCH_F64, RID_SKETCH_F32, RID_SKETCH_BF16, RID_SKETCH_FP8 = 0, 1, 2, 3
RID_COPY, RID_BORROW = 0, 1
RID_TILE_AUTO, RID_TILE_NARROW, RID_TILE_WIDE = 0, 1, 2
RID_COEFF_ALG4, RID_COEFF_BEST4 = 0, 1
RID_GRAM_AUTO, RID_GRAM_EXACT, RID_GRAM_SPLIT = 0, 1, 2
RID_HOST, RID_DEVICE = 0, 1
RID_UPD_SKIPPED, RID_UPD_RANK_DEFICIENT, RID_UPD_PINV_TRUNCATED = 1, 2, 4


class rid_config(C.Structure):
    _fields_ = [
        ("m", C.c_int64), ("ell", C.c_int32), ("k", C.c_int32), ("t", C.c_int32),
        ("data_dtype", C.c_int32), ("sketch_prec", C.c_int32),
        ("omega_seed", C.c_uint64), ("select_seed", C.c_uint64),
        ("delta", C.c_double), ("eps", C.c_double), ("c_sample", C.c_double), ("ridge_floor", C.c_double),
        ("hutch_n1", C.c_int32), ("hutch_n2", C.c_int32), ("lookahead", C.c_int32), ("sketch_tile", C.c_int32),
        ("n_max", C.c_int64), ("coeff_mode", C.c_int32), ("gram_mode", C.c_int32),
    ]


class rid_error(C.Structure):
    _fields_ = [("E2", C.c_double), ("E_abs", C.c_double), ("rel", C.c_double), ("F", C.c_double),
                ("n_obs", C.c_int64), ("update", C.c_int64)]


class rid_update(C.Structure):
    _fields_ = [("update", C.c_int64), ("n_obs", C.c_int64), ("count", C.c_int64),
                ("F", C.c_double), ("sk2", C.c_double), ("lam", C.c_double),
                ("E2", C.c_double), ("tr_est", C.c_double), ("gpp", C.c_double),
                ("term1", C.c_double), ("h", C.c_double), ("corr", C.c_double),
                ("n_pruned", C.c_int32), ("n_filled", C.c_int32), ("n_occupied", C.c_int32),
                ("flags", C.c_int32)]


class rid_info(C.Structure):
    _fields_ = [("n_pushed", C.c_int64), ("n_sketched", C.c_int64), ("n_updates", C.c_int64),
                ("release_watermark", C.c_int64), ("failed", C.c_int32), ("finalized", C.c_int32),
                ("last_status", C.c_int32), ("reserved0", C.c_int32), ("device_bytes", C.c_int64)]


class rid_profile(C.Structure):
    _fields_ = [("sketch_ms", C.c_double), ("sketch_launches", C.c_int64), ("sketch_bytes", C.c_double),
                ("reduce_ms", C.c_double), ("update_ms", C.c_double), ("updates", C.c_int64),
                ("gram_ms", C.c_double), ("gram_bytes", C.c_double), ("coeff_ms", C.c_double),
                ("pool_copy_bytes", C.c_double), ("gram_launches", C.c_int64)]


RID_BATCH_NO_GRAPH, RID_BATCH_NO_TUNE = 1, 2


class rid_batch_info(C.Structure):
    _fields_ = [("ns", C.c_int32), ("failed", C.c_int32), ("rounds", C.c_int64), ("graph_launches", C.c_int64),
                ("graph_instantiations", C.c_int64), ("graph_updates", C.c_int64), ("slab_rows", C.c_int64),
                ("tuned", C.c_int32), ("wide", C.c_int32), ("tune_ms", C.c_double)]


# name -> (restype, argtypes); every function declared in include/rid.h
SIGNATURES = {
    "rid_config_default": (C.c_int, [C.POINTER(rid_config)]),
    "rid_init_stream": (C.c_int, [C.POINTER(rid_config), C.c_void_p, C.POINTER(C.c_void_p)]),
    "rid_push_snapshots": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_uint32]),
    "rid_flush": (C.c_int, [C.c_void_p]),
    "rid_finalize": (C.c_int, [C.c_void_p]),
    "rid_reset": (C.c_int, [C.c_void_p]),
    "rid_select": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32)]),
    "rid_coefficients": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.POINTER(C.c_int64), C.c_uint32]),
    "rid_error_estimate": (C.c_int, [C.c_void_p, C.POINTER(rid_error)]),
    "rid_reconstruct": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_int64]),
    "rid_get_info": (C.c_int, [C.c_void_p, C.POINTER(rid_info)]),
    "rid_get_update": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(rid_update), C.c_void_p, C.c_void_p, C.c_void_p]),
    "rid_destroy": (C.c_int, [C.c_void_p]),
    "rid_status_string": (C.c_char_p, [C.c_int]),
    "rid_last_error": (C.c_int, [C.c_void_p, C.c_char_p, C.c_size_t]),
    "rid_get_coeff_choice": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.POINTER(C.c_int32)]),
    "rid_debug_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.POINTER(C.c_int64), C.c_void_p, C.c_void_p]),
    "rid_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "rid_profile_read": (C.c_int, [C.c_void_p, C.POINTER(rid_profile)]),
    "rid_omega_block": (C.c_int, [C.c_int32, C.c_uint64, C.c_int32, C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]),
    "rid_sketch_columns": (C.c_int, [C.c_int32, C.c_uint64, C.c_int32, C.c_int64, C.c_void_p, C.c_int64, C.c_int32,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rid_sketch_columns_noalloc": (C.c_int, [C.c_int32, C.c_uint64, C.c_int32, C.c_int64, C.c_void_p, C.c_int64,
                                             C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rid_init_batch": (C.c_int, [C.c_int32, C.POINTER(rid_config), C.c_void_p, C.c_uint32, C.POINTER(C.c_void_p)]),
    "rid_push_batch": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                 C.c_uint32]),
    "rid_finalize_batch": (C.c_int, [C.c_void_p]),
    "rid_reset_batch": (C.c_int, [C.c_void_p]),
    "rid_batch_stream": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    "rid_batch_get_info": (C.c_int, [C.c_void_p, C.POINTER(rid_batch_info)]),
    "rid_batch_last_error": (C.c_int, [C.c_void_p, C.c_char_p, C.c_size_t]),
    "rid_batch_tune_result": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_double)]),
    "rid_destroy_batch": (C.c_int, [C.c_void_p]),
    "rid_batch_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "rid_batch_profile_read": (C.c_int, [C.c_void_p, C.POINTER(rid_profile)]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2405_16076_amd.build` (there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class RIDError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{lib().rid_status_string(status).decode()}: {message}")
        self.status = status


def check(status, handle=None, batch=None):
    if status != RID_OK:
        buf = C.create_string_buffer(512)
        if batch is not None:
            lib().rid_batch_last_error(batch, buf, 512)
        else:
            lib().rid_last_error(handle, buf, 512)
        raise RIDError(status, buf.value.decode(errors="replace"))
