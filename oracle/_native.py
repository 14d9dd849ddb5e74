"""Loader of the oracle's C helper (test infrastructure only).

oracle/eigref.c is compiled with gcc into oracle/liboracle_eigref.so, by
__graft_entry__.build() or, when missing or older than its source, here on first use.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "eigref.c")
LIB = os.path.join(HERE, "liboracle_eigref.so")
_lock = threading.Lock()
_lib = None


def build() -> str:
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build()
            l = ctypes.CDLL(LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            l.oracle_eig_refine.restype = ctypes.c_int
            l.oracle_eig_refine.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_double, ctypes.c_double, dp, dp, dp, dp, dp]
            _lib = l
    return _lib


def eig_refine(ops, xr: np.ndarray, wr: np.ndarray, lam: np.ndarray, s: np.ndarray):
    """One extended-precision refinement step (see eigref.c); returns new (lam, S)."""
    n = lam.size
    lo = np.array(lam, dtype=np.float64, copy=True)
    so = np.array(s, dtype=np.float64, copy=True, order="C")
    xr = np.ascontiguousarray(xr, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    md = np.ascontiguousarray(ops.M, dtype=np.float64)
    off = 1 if ops.bc == "dirichlet" else 0
    per = 1 if ops.bc == "periodic" else 0
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib().oracle_eig_refine(n, ops.k, ops.ne, off, per, ops.a, ops.b, xr.ctypes.data_as(dp), wr.ctypes.data_as(dp),
                                 md.ctypes.data_as(dp), lo.ctypes.data_as(dp), so.ctypes.data_as(dp))
    if st != 0:
        raise MemoryError("oracle_eig_refine: allocation failed")
    return lo, so
