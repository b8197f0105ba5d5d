"""ctypes loader for oracle/cmax.c (test infrastructure only; see oracle/__init__).

``build()`` compiles the C file with gcc into ``oracle/_cmax.so``; the loader
compiles it on first use if the library is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cmax.c")
_LIB = os.path.join(_HERE, "_cmax.so")
_lib = None


def build() -> str:
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", _LIB, _SRC], check=True)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_max_sqdist.restype = ctypes.c_double
        lib.oracle_max_sqdist.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_int32]
        _lib = lib
    return _lib


def max_sqdist(x: np.ndarray, y: np.ndarray) -> float:
    """max_ij ||x_i - y_j||^2 for FP32 clouds, exact FP64 arithmetic."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    assert x.shape[1] == y.shape[1]
    return float(_load().oracle_max_sqdist(x.ctypes.data, y.ctypes.data, x.shape[0], y.shape[0],
                                           x.shape[1]))
