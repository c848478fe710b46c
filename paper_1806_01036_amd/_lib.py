"""ctypes binding of libborth.so (include/borth.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch provides device memory (tensors) and the current stream.
If the library has not been built, every call raises -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libborth.so"

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double


class borth_opts(ctypes.Structure):
    _fields_ = [("gram", _int), ("fact", _int), ("passes", _int), ("sched", _int),
                ("shift", _dbl), ("flags", ctypes.c_uint)]


class borth_info(ctypes.Structure):
    _fields_ = [("status", _int), ("failed_pass", _int), ("failed_pivot", _int),
                ("passes_run", _int), ("orth_est", _dbl), ("kappa_est", _dbl),
                ("escalation", _int), ("svqb_lifted", _int)]


class borth_block(ctypes.Structure):
    _fields_ = [("m", _i64), ("k", _int), ("X", _vp), ("ldx", _i64), ("Y", _vp),
                ("ldy", _i64), ("ky", _int), ("Q", _vp), ("ldq", _i64), ("R", _vp),
                ("C", _vp)]


class borth_iter_info(ctypes.Structure):
    _fields_ = [("converged", _int), ("passes_run", _int), ("c_norm", _dbl), ("r_dev", _dbl),
                ("rank", _int)]


EXPORTS = {
    "borth_default_opts": ([ctypes.POINTER(borth_opts)], None),
    "borth_create": ([ctypes.POINTER(_vp), _int, _vp], _int),
    "borth_destroy": ([_vp], _int),
    "borth_set_stream": ([_vp, _vp], _int),
    "borth_status_string": ([_int], ctypes.c_char_p),
    "borth_last_error": ([_vp], ctypes.c_char_p),
    "borth_get_info": ([_vp, ctypes.POINTER(borth_info)], _int),
    "borth_gram": ([_vp, _i64, _int, _vp, _i64, _int, _int, _vp, _i64, _int, _vp, _vp], _int),
    "borth_factor": ([_vp, _int, _int, _vp, _vp, _int, _dbl, _vp, _vp, _vp,
                      ctypes.POINTER(borth_info)], _int),
    "borth_update": ([_vp, _i64, _int, _int, _vp, _i64, _vp, _i64, _int, _vp, _vp, _int, _vp,
                      _i64], _int),
    "borth_orthonormalize": ([_vp, _i64, _int, _int, _vp, _i64, _vp, _i64, _int, _vp, _i64,
                              _vp, _vp, ctypes.POINTER(borth_opts),
                              ctypes.POINTER(borth_info)], _int),
    "borth_stream_probe": ([_vp, _int, _vp, _vp, _i64, _int, ctypes.POINTER(_dbl),
                            ctypes.POINTER(_int)], _int),
    "borth_valu_probe": ([_vp, _int, _vp, _i64, ctypes.POINTER(_dbl), ctypes.POINTER(_int)],
                          _int),
    "borth_orthonormalize_noalloc": ([_vp, _i64, _int, _int, _vp, _i64, _vp, _i64, _int, _vp,
                                      _i64, _vp, _vp, ctypes.POINTER(borth_opts),
                                      ctypes.POINTER(borth_info)], _int),
    "borth_orthonormalize_dd": ([_vp, _i64, _int, _vp, _vp, _i64, _vp, _i64, _int, _vp, _vp, _i64,
                                 _vp, _vp, ctypes.POINTER(borth_opts), ctypes.POINTER(borth_info)],
                                _int),
    "borth_orthonormalize_iter": ([_vp, _i64, _int, _vp, _i64, _vp, _i64, _int, _vp, _i64,
                                   _vp, _vp, ctypes.POINTER(borth_opts), _dbl, _int,
                                   ctypes.POINTER(borth_iter_info), ctypes.POINTER(borth_info)],
                                  _int),
    "borth_orthonormalize_iter_b": ([_vp, _i64, _int, _vp, _i64, _vp, _i64, _int, _vp, _vp,
                                     _i64, _vp, _vp, ctypes.POINTER(borth_opts), _dbl, _int,
                                     ctypes.POINTER(borth_iter_info), ctypes.POINTER(borth_info)],
                                    _int),
    "borth_batch_orthonormalize": ([_vp, _int, ctypes.POINTER(borth_block),
                                    ctypes.POINTER(borth_opts), ctypes.POINTER(borth_info)],
                                   _int),
    "borth_autotune": ([_vp, ctypes.c_char_p, _int], _int),
    "borth_autotune_load": ([_vp, ctypes.c_char_p], _int),
    "borth_set_profiling": ([_vp, _int], _int),
    "borth_kernel_time": ([_vp, _int, ctypes.POINTER(_dbl), ctypes.POINTER(_int)], _int),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libborth.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1806_01036_amd.build` (there is no CPU fallback)")
        lib = ctypes.CDLL(str(LIB_PATH))
        for name, (args, res) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib
