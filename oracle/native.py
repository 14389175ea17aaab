"""ctypes binding of the oracle's C part (test infrastructure)."""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        L.or_fps.restype = ctypes.c_int
        L.or_fps.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        L.or_flood.restype = ctypes.c_int
        L.or_flood.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        L.or_flood_random.restype = ctypes.c_int
        L.or_flood_random.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int]
        L.or_random_weights.restype = None
        L.or_random_weights.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                        ctypes.c_void_p]
        L.or_philox4x64_10.restype = None
        L.or_philox4x64_10.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.or_max_threads.restype = ctypes.c_int
        L.or_count_samples.restype = ctypes.c_int64
        L.or_count_samples.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
        _lib = L
    return _lib


def threads(n=None) -> int:
    if n:
        return int(n)
    env = os.environ.get("OMP_NUM_THREADS")
    if env:
        return int(env)
    return lib().or_max_threads()


def ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)
