"""Build and load the oracle's plain-C helpers (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ilu0.c")
_LIB = os.path.join(_HERE, "_oracle_c.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle's C sources with gcc (seconds)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        i64, p = ctypes.c_int64, ctypes.c_void_p
        _lib.oracle_ilu0_factor.argtypes = [i64, p, p, p, p]
        _lib.oracle_ilu0_factor.restype = i64
        _lib.oracle_ilu0_solve.argtypes = [i64, p, p, p, p, p, p]
        _lib.oracle_ilu0_solve.restype = None
    return _lib
