"""Loader for the plain-C oracle loops (``modmatmul_ref.c``).

``build()`` compiles the file with gcc into ``oracle/_oracle_ref.so``; the
loader compiles on first use when the library is missing.  Test
infrastructure only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "modmatmul_ref.c")
_LIB = os.path.join(_HERE, "_oracle_ref.so")
_lock = threading.Lock()
_lib = None
_failed = False


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib, _failed
    with _lock:
        if _lib is not None or _failed:
            return _lib
        try:
            if not os.path.exists(_LIB):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            I = ctypes.c_int64
            lib.oracle_modmatmul.argtypes = [P, P, P, I, I, I, ctypes.c_uint32]
            lib.oracle_modmatmul.restype = None
            lib.oracle_exact_matmul.argtypes = [P, P, P, I, I, I]
            lib.oracle_exact_matmul.restype = None
            lib.oracle_set_threads.argtypes = [ctypes.c_int]
            lib.oracle_set_threads.restype = None
            lib.oracle_num_threads.argtypes = []
            lib.oracle_num_threads.restype = ctypes.c_int
            _lib = lib
        except Exception:
            _failed = True
            _lib = None
        return _lib


def available() -> bool:
    return _load() is not None


def num_threads() -> int:
    lib = _load()
    return int(lib.oracle_num_threads()) if lib is not None else 1


def set_threads(n: int) -> None:
    """Threads of the OpenMP loops from now on (for single-core timings)."""
    lib = _load()
    if lib is not None:
        lib.oracle_set_threads(int(n))


def modmatmul(a: np.ndarray, b: np.ndarray, p: int) -> np.ndarray:
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    m, k = a.shape
    k2, n = b.shape
    assert k == k2
    c = np.empty((m, n), dtype=np.uint32)
    lib.oracle_modmatmul(a.ctypes.data, b.ctypes.data, c.ctypes.data, m, n, k, int(p))
    return c


def exact_matmul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.int64)
    b = np.ascontiguousarray(b, dtype=np.int64)
    m, k = a.shape
    k2, n = b.shape
    assert k == k2
    c = np.empty((m, n), dtype=np.int64)
    lib.oracle_exact_matmul(a.ctypes.data, b.ctypes.data, c.ctypes.data, m, n, k)
    return c
