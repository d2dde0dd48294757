"""ctypes binding of libhbi.so (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhbi.so")

HBI_OK, HBI_ERR_ARG, HBI_ERR_STATE, HBI_ERR_OOM, HBI_ERR_HIP, HBI_ERR_NUMERIC = range(6)
HBI_F64, HBI_F32 = 0, 1
STATUS_NAMES = {0: "HBI_OK", 1: "HBI_ERR_ARG", 2: "HBI_ERR_STATE", 3: "HBI_ERR_OOM",
                4: "HBI_ERR_HIP", 5: "HBI_ERR_NUMERIC"}


class hbi_tables(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("ncell", ctypes.c_int32 * 3),
        ("origin", ctypes.c_double * 3),
        ("h", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("nterms", ctypes.c_int32),
        ("nI", ctypes.c_int32),
        ("nbox", ctypes.c_int32 * 3),
        ("box_origin", ctypes.c_double * 3),
        ("box_size", ctypes.c_double),
        ("tau2", ctypes.POINTER(ctypes.c_double)),
        ("v0", ctypes.POINTER(ctypes.c_double)),
        ("v1", ctypes.POINTER(ctypes.c_double)),
        ("slowness", ctypes.POINTER(ctypes.c_double)),
    ]


class hbi_build_opts(ctypes.Structure):
    _fields_ = [
        ("chi", ctypes.c_double),
        ("leaf_size", ctypes.c_int32),
        ("neighbor_radius", ctypes.c_double),
        ("band_width", ctypes.c_int32),
        ("workspace_bytes", ctypes.c_int64),
    ]


class HBIError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

class hbi_medium2d(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 2), ("origin", ctypes.c_double * 2),
                ("spacing", ctypes.c_double), ("n2", ctypes.POINTER(ctypes.c_double)),
                ("taylor", ctypes.POINTER(ctypes.c_double))]


# (name, restype, argtypes) for every function declared in include/hbi.h
SIGNATURES = [
    ("hbi_create", ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    ("hbi_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("hbi_set_stream", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("hbi_load_tables", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(hbi_tables)]),
    ("hbi_load_tables_from", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double]),
    ("hbi_set_inclusion", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]),
    ("hbi_set_build_opts", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(hbi_build_opts)]),
    ("hbi_build", ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, ctypes.c_int]),
    ("hbi_apply", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_int32, ctypes.c_int64]),
    ("hbi_apply_adjoint", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_int64]),
    ("hbi_apply_noalloc", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_int64]),
    ("hbi_apply_batched", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int64)]),
    ("hbi_entries", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_void_p]),
    ("hbi_set_profiling", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("hbi_get_profile", ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int64]),
    ("hbi_get_info", ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int64]),
    ("hbi_last_error", ctypes.c_char_p, [ctypes.c_void_p]),
    ("hbi_tabulate", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(hbi_medium2d), ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]),
]


def load(path: str = LIB_PATH):
    """Load libhbi.so; raises loudly when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libhbi.so not found at {path}: build it first with "
            "`python -m paper_2210_02698_amd.build` (there is no fallback path)")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status, ctx=None):
    if status != HBI_OK:
        lib = load()
        msg = lib.hbi_last_error(ctx)
        raise HBIError(status, msg.decode() if msg else "")
