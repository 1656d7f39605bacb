"""ctypes declarations of include/petar.h (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpetar.so")

PETAR_OK = 0
PETAR_E_INVALID = -1
PETAR_E_NOMEM = -2
PETAR_E_HIP = -3
PETAR_E_NB_OVERFLOW = -4
PETAR_E_STATE = -5
PETAR_E_NODEVICE = -6
PETAR_E_INTERNAL = -7

PETAR_MIXED = 0
PETAR_FP64 = 1
PETAR_NO_DEVICE = -1

STATUS_NAMES = {
    PETAR_OK: "PETAR_OK", PETAR_E_INVALID: "PETAR_E_INVALID", PETAR_E_NOMEM: "PETAR_E_NOMEM",
    PETAR_E_HIP: "PETAR_E_HIP", PETAR_E_NB_OVERFLOW: "PETAR_E_NB_OVERFLOW",
    PETAR_E_STATE: "PETAR_E_STATE", PETAR_E_NODEVICE: "PETAR_E_NODEVICE",
    PETAR_E_INTERNAL: "PETAR_E_INTERNAL",
}


class petar_params(ctypes.Structure):
    _fields_ = [("G", ctypes.c_double), ("precision", ctypes.c_int), ("i_per_lane", ctypes.c_int),
                ("record_counts", ctypes.c_int), ("workspace_cap", ctypes.c_int64)]


class petar_nblist(ctypes.Structure):
    _fields_ = [("offsets_dev", ctypes.c_void_p), ("idx_dev", ctypes.c_void_p),
                ("capacity", ctypes.c_int64), ("required", ctypes.c_int64)]


class petar_stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_nodes", ctypes.c_int64), ("n_leaves", ctypes.c_int64),
                ("n_groups", ctypes.c_int64), ("max_level", ctypes.c_int64),
                ("inter_pc", ctypes.c_int64), ("inter_far", ctypes.c_int64),
                ("inter_near", ctypes.c_int64), ("nb_total", ctypes.c_int64),
                ("ms_build", ctypes.c_double), ("ms_force", ctypes.c_double),
                ("ms_force_kernel", ctypes.c_double), ("ms_nb", ctypes.c_double),
                ("ms_graph", ctypes.c_double), ("workspace_bytes", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class petar_tuned(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int), ("group_size", ctypes.c_int),
                ("i_per_lane", ctypes.c_int), ("ms", ctypes.c_double)]


class petar_art_set(ctypes.Structure):
    _fields_ = [("pos_dev", ctypes.c_void_p), ("mass_dev", ctypes.c_void_p),
                ("r_in_dev", ctypes.c_void_p), ("r_out_dev", ctypes.c_void_p),
                ("r_search_dev", ctypes.c_void_p), ("src_dev", ctypes.c_void_p),
                ("n_out", ctypes.c_int64), ("target_dev", ctypes.c_void_p)]


# (name, restype, argtypes) of every exported entry point
_P = ctypes.c_void_p
_D = ctypes.c_double
_I64 = ctypes.c_int64
_INT = ctypes.c_int
SIGNATURES = [
    ("petar_create", _INT, [ctypes.POINTER(_P), _INT, _P]),
    ("petar_destroy", _INT, [_P]),
    ("petar_set_params", _INT, [_P, ctypes.POINTER(petar_params)]),
    ("petar_get_params", _INT, [_P, ctypes.POINTER(petar_params)]),
    ("petar_changeover_radii", _INT, [_P, _P, _P, _I64, _D, _D, _D, _D, _P, _P, _P]),
    ("petar_tree_build", _INT, [_P, _P, _P, _I64, _D, _INT]),
    ("petar_batch_build", _INT, [_P, _INT, ctypes.POINTER(_I64), _P, _P, _D, _INT]),
    ("petar_force_long", _INT, [_P, _INT, _P, _P, _P, _P, _P, ctypes.POINTER(petar_nblist)]),
    ("petar_force_long_kick", _INT, [_P, _INT, _P, _P, _P, _P, _P, ctypes.POINTER(petar_nblist),
                                     _P, _D]),
    ("petar_step_graph", _INT, [_P, _INT, ctypes.POINTER(_I64), _P, _P, _I64, _D, _INT, _INT,
                                _P, _P, _P, _P, _P, ctypes.POINTER(petar_nblist)]),
    ("petar_copy_counts", _INT, [_P, _P]),
    ("petar_get_stats", _INT, [_P, ctypes.POINTER(petar_stats)]),
    ("petar_autotune", _INT, [_P, _P, _P, _I64, _D, _P, _P, _P, ctypes.c_char_p,
                              ctypes.POINTER(petar_tuned)]),
    ("petar_autotune_lookup", _INT, [_P, _I64, _D, ctypes.c_char_p, ctypes.POINTER(petar_tuned)]),
    ("petar_autotune_batch", _INT, [_P, _INT, ctypes.POINTER(_I64), _P, _P, _D, _P, _P, _P,
                                    ctypes.c_char_p, ctypes.POINTER(petar_tuned)]),
    ("petar_autotune_lookup_batch", _INT, [_P, _I64, _INT, _D, ctypes.c_char_p,
                                           ctypes.POINTER(petar_tuned)]),
    ("petar_nb_filter", _INT, [_P, _I64, _P, _P, _P, _P, _D, _P, _P,
                               ctypes.POINTER(petar_nblist)]),
    ("petar_set_targets", _INT, [_P, _P]),
    ("petar_clusters", _INT, [_P, _I64, _P, _P, _P, _P, _P, ctypes.POINTER(_I64)]),
    ("petar_clusters_noalloc", _INT, [_P, _I64, _P, _P, _P, _P, _P, ctypes.POINTER(_I64)]),
    ("petar_groups", _INT, [_P, _I64, _P, _P, _P, _P, _D, _P, _P, _P, _P, _P,
                            ctypes.POINTER(_I64), _P, _I64, ctypes.POINTER(_I64)]),
    ("petar_kick", _INT, [_P, _I64, _P, _P, _D]),
    ("petar_artificial_make", _INT, [_P, _I64, _P, _P, _P, _P, _P, _P, _I64, _P, _INT, _D,
                                     ctypes.POINTER(petar_art_set), _P, _P]),
    ("petar_tidal_fit", _INT, [_P, _INT, _I64, _P, _I64, _P, _P, _I64, _P, _P, _P, _P, _P, _P]),
    ("petar_tidal_eval", _INT, [_P, _INT, _I64, _P, _P, _I64, _P, _P, _P, _P]),
    ("petar_last_error", ctypes.c_char_p, [_P]),
    ("petar_status_string", ctypes.c_char_p, [_INT]),
]

_lib = None


def load(path: str = LIB_PATH):
    """Load libpetar.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(
                "libpetar.so is missing (%s): build it with "
                "`python paper_2006_16560_amd/build.py` (hipcc, gfx950)" % path)
        lib = ctypes.CDLL(path)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
