"""ORACLE (test infrastructure): build and load the plain-C part of the oracle.

Only tests, the smoke check and the benchmark's CPU-baseline leg use this.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile cd_oracle.c with gcc (-O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-ffp-contract=off",
               SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(LIB)
        d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        P = ctypes.c_void_p
        L.orc_boys_f0.argtypes = [d]
        L.orc_boys_f0.restype = d
        L.orc_eri4.argtypes = [P, d, P, d, P, d, P, d]
        L.orc_eri4.restype = d
        L.orc_eri_matrix.argtypes = [i32, P, P, P]
        L.orc_eri_matrix.restype = None
        L.orc_eri_columns.argtypes = [i32, P, P, i64, P, P]
        L.orc_eri_columns.restype = None
        L.orc_eri_diagonal.argtypes = [i32, P, P, P]
        L.orc_eri_diagonal.restype = None
        L.orc_pivoted_cd.argtypes = [i64, P, i32, P, P, d, d, d, i64, i64, P, P, P, P, P, P, i32]
        L.orc_pivoted_cd.restype = ctypes.c_int
        _lib = L
    return _lib
