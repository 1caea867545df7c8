"""Build and load the oracle's plain-C FP64 solver (test infrastructure)."""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "fd_oracle.c")
LIB = os.path.join(_HERE, "_fd_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile fd_oracle.c with gcc -O2 (IEEE semantics, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_energy_gradient.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                             dp, dp, dp, dp]
        L.oracle_energy_gradient.restype = None
        L.oracle_apply_operator.argtypes = L.oracle_energy_gradient.argtypes
        L.oracle_apply_operator.restype = None
        L.oracle_solve.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int, dp, dp, dp,
                                   ctypes.c_int, ip, ip, ctypes.c_int, ctypes.c_int,
                                   dp, dp, ctypes.c_int, ip, ip, dp, dp, dp, dp,
                                   ctypes.c_int]
        L.oracle_solve.restype = ctypes.c_int
        _lib = L
    return _lib
