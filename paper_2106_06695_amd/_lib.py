"""ctypes loader for libsimplexgp.so with the signatures of include/simplexgp.h."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsimplexgp.so")

_lib = None


class Opts(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("kernel", ctypes.c_int32), ("blur", ctypes.c_int32),
                ("outputscale", ctypes.c_float), ("load_factor", ctypes.c_float),
                ("solve_rows", ctypes.c_int64)]


# name -> (restype, argtypes), one entry per declaration in include/simplexgp.h
_P, _I32, _I64, _F, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
# sgp_set_allocator's hooks: alloc(bytes, stream) -> device pointer, free(ptr, stream)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
SIGNATURES = {
    "sgp_opts_default": (None, [_P]),
    "lattice_build": (ctypes.c_int, [_P, _I64, _I32, _P, _P, _P, _P]),
    "lattice_mvm": (ctypes.c_int, [_P, _P, _I32, _P, _P]),
    "lattice_mvm_noalloc": (ctypes.c_int, [_P, _P, _I32, _P, _P]),
    "cg_solve": (ctypes.c_int, [_P, _P, _I32, _F, _F, _I32, _P, _P, _P, _P]),
    "lattice_mvm_grad": (ctypes.c_int, [_P, _P, _P, _P, _I32, _P, _P, _P]),
    "lattice_info": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "lattice_export": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "lattice_free": (None, [_P]),
    "sgp_last_error": (ctypes.c_char_p, []),
    "sgp_set_allocator": (ctypes.c_int, [_P, _P]),  # ALLOC_FN / FREE_FN pointers, or NULL
    "sgp_cache_info": (ctypes.c_int, [_P, _P]),
    "sgp_debug_inject_oom": (ctypes.c_int, [_I32]),
    "sgp_cg_graph_enable": (ctypes.c_int, [ctypes.c_int]),
    "sgp_blur_fuse_enable": (ctypes.c_int, [ctypes.c_int]),
    "sgp_blur_seq_bytes": (ctypes.c_int64, [ctypes.c_int64]),
    "sgp_cg_fuse_enable": (ctypes.c_int, [ctypes.c_int]),
    "sgp_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sgp_autotune_reset": (ctypes.c_int, []),
    "sgp_autotune_build": (ctypes.c_int, [_P, _I64, _I32, _P, _P, _I32, _P, _P, _P, _P]),
    "sgp_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "sgp_profile_reset": (ctypes.c_int, []),
    "sgp_profile_kinds": (ctypes.c_int, []),
    "sgp_profile_name": (ctypes.c_char_p, [ctypes.c_int]),
    "sgp_profile_read": (ctypes.c_int, [ctypes.c_int, _P, _P]),
}


def load():
    """Load the built library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
