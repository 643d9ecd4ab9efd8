"""ctypes binding of libparis.so (include/paris.h). Argument marshalling only: every step of the
search runs in the library's HIP kernels. PyTorch supplies device memory and streams."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libparis.so")

PARIS_OK, PARIS_EINVAL, PARIS_ENOMEM, PARIS_ENODEV, PARIS_EHIP, PARIS_EOVERFLOW, PARIS_ESTATE = \
    0, -1, -2, -3, -4, -5, -6
LEAF_ROOT16, LEAF_EQUAL_COUNT, LEAF_ADS = 0, 1, 2


class ParisConfig(ctypes.Structure):
    _fields_ = [("segments", ctypes.c_int32), ("card_bits", ctypes.c_int32),
                ("leaf_mode", ctypes.c_int32), ("n_leaves", ctypes.c_int32),
                ("seed_cap", ctypes.c_int32), ("leaf_cap", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class ParisStats(ctypes.Structure):
    _fields_ = [("lb_survivors", ctypes.c_int64), ("refined", ctypes.c_int64),
                ("abandoned", ctypes.c_int64), ("bsf_updates", ctypes.c_int64),
                ("resolved", ctypes.c_int64), ("seed_index", ctypes.c_int64),
                ("seed_dist", ctypes.c_double), ("seed_lo", ctypes.c_int64),
                ("seed_hi", ctypes.c_int64), ("words_read", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ParisLayout(ctypes.Structure):
    _fields_ = [("sax_dev", ctypes.c_void_p), ("keys_dev", ctypes.c_void_p),
                ("perm_dev", ctypes.c_void_p), ("roff_dev", ctypes.c_void_p),
                ("n_series", ctypes.c_int64), ("length", ctypes.c_int32),
                ("leaf_mode", ctypes.c_int32), ("n_leaves", ctypes.c_int32),
                ("seed_cap", ctypes.c_int32), ("scan_threads", ctypes.c_int32),
                ("scan_blocks_per_cu", ctypes.c_int32), ("scan_unroll", ctypes.c_int32),
                ("tree_nodes_dev", ctypes.c_void_p), ("n_tree_nodes", ctypes.c_int64),
                ("tree_max_leaf", ctypes.c_int64), ("screen_rows", ctypes.c_int32),
                ("screen_blocks_per_cu", ctypes.c_int32), ("screen_subtiles", ctypes.c_int32),
                ("screen_mfma", ctypes.c_int32)]


class ParisQueryInfo(ctypes.Structure):
    _fields_ = [("paa", ctypes.c_double * 16), ("sym", ctypes.c_uint8 * 16),
                ("root", ctypes.c_uint32), ("pad", ctypes.c_uint32), ("k64", ctypes.c_uint64),
                ("win_lo", ctypes.c_int64), ("win_hi", ctypes.c_int64)]


class ParisAdam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


# (name, restype, argtypes) for every entry point declared in include/paris.h
_P, _I64, _I32, _F32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float
SIGNATURES = [
    ("paris_default_config", ctypes.c_int, [ctypes.POINTER(ParisConfig)]),
    ("paris_workspace_size", ctypes.c_int, [_I64, _I32, ctypes.POINTER(ParisConfig),
                                            ctypes.POINTER(ctypes.c_size_t)]),
    ("paris_build", ctypes.c_int, [_P, _I64, _I32, ctypes.POINTER(ParisConfig), _P, ctypes.c_size_t,
                                   _P, ctypes.POINTER(_P)]),
    ("paris_get_layout", ctypes.c_int, [_P, ctypes.POINTER(ParisLayout)]),
    ("paris_query_exact", ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ParisStats), _P]),
    ("paris_query_knn", ctypes.c_int, [_P, _P, _I32, _P, _P, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ParisStats), _P]),
    ("paris_query_exact_noalloc", ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_int64),
                                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ParisStats), _P]),
    ("paris_query_batch", ctypes.c_int, [_P, _P, _I64, _P, _P, ctypes.POINTER(ParisStats), _P]),
    ("paris_query_batch_multi", ctypes.c_int, [_P, _I32, _P, _P, _P, _P, ctypes.POINTER(ParisStats), _P]),
    ("paris_query_info_get", ctypes.c_int, [_P, _P, ctypes.POINTER(ParisQueryInfo), _P, _P]),
    ("paris_lb_scan", ctypes.c_int, [_P, _P, _F32, _P, _P, _I64, ctypes.POINTER(ctypes.c_int64), _P]),
    ("paris_batch_workspace_size", ctypes.c_int, [_P, _I32, ctypes.POINTER(ctypes.c_size_t)]),
    ("paris_batch_attach", ctypes.c_int, [_P, _P, ctypes.c_size_t, _I32, _P]),
    ("paris_screen_dots", ctypes.c_int, [_P, _P, _I32, _P, _P]),
    ("paris_batch_screen_tiles", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), _I32]),
    ("paris_block_bound_bits", ctypes.c_int, [_P, _P, _P, _I32, _I32, _P, _P]),
    ("paris_set_bsf_sharing", ctypes.c_int, [_P, _I32]),
    ("paris_set_timing", ctypes.c_int, [_P, _I32]),
    ("paris_get_timing", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    ("paris_get_batch_timing", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    ("paris_free", ctypes.c_int, [_P]),
    ("paris_mlp_param_count", ctypes.c_int, [_I32, ctypes.POINTER(ctypes.c_int64)]),
    ("paris_mlp_workspace_size", ctypes.c_int, [_I32, _I32, ctypes.POINTER(ctypes.c_int64)]),
    ("paris_mlp_create", ctypes.c_int, [_I32, _I32, _P, _I64, ctypes.POINTER(_P)]),
    ("paris_mlp_set_params", ctypes.c_int, [_P, _P, _P]),
    ("paris_mlp_get_params", ctypes.c_int, [_P, _P, _P]),
    ("paris_query_features", ctypes.c_int, [_P, _I64, _I32, _P, _P]),
    ("paris_mlp_forward", ctypes.c_int, [_P, _P, _I64, _P, _P]),
    ("paris_mlp_top_leaves", ctypes.c_int, [_P, _P, _I64, _P, _P]),
    ("paris_mlp_grad", ctypes.c_int, [_P, _P, _P, _P, _I64, _P, _P, _P]),
    ("paris_mlp_train_step", ctypes.c_int, [_P, _P, _P, _P, _I64, ctypes.POINTER(ParisAdam), _P, _P]),
    ("paris_mlp_apply", ctypes.c_int, [_P, _P, ctypes.POINTER(ParisAdam), _P]),
    ("paris_mlp_free", ctypes.c_int, [_P]),
    ("paris_leaf_of", ctypes.c_int, [_P, _P, _I64, _P, _P]),
    ("paris_set_seed_model", ctypes.c_int, [_P, _P, _I32]),
    ("paris_host_alloc", ctypes.c_int, [ctypes.c_size_t, ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    ("paris_host_free", ctypes.c_int, [_P]),
    ("paris_status_string", ctypes.c_char_p, [ctypes.c_int]),
]

_lib = None


def load_library():
    """Load libparis.so; raises ImportError if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class ParisError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = load_library().paris_status_string(status).decode()
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)


def check(status: int, what: str = "") -> None:
    if status != PARIS_OK:
        raise ParisError(status, what)
