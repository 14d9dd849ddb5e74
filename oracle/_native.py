"""Loader of the oracle's C helper (test infrastructure only).

oracle/eigjac.c is compiled with gcc into oracle/liboracle_eigjac.so, by
__graft_entry__.build() or, when missing or older than its source, here on first use.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "eigjac.c")
LIB = os.path.join(HERE, "liboracle_eigjac.so")
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
            ci = ctypes.c_int
            l.oracle_eig_jacobi.restype = ci
            l.oracle_eig_jacobi.argtypes = [ci, ci, ci, ci, ci, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                            dp, dp, dp]
            _lib = l
    return _lib


def eig_jacobi(ops, q0: np.ndarray):
    """Eigenpairs of the axis ops by long-double cyclic Jacobi started from q0
    (see eigjac.c); returns (lam, S), ascending, S^T M S = I."""
    import mpmath

    from .sem_oracle import element_matrices_hp
    n = q0.shape[0]
    (khi, klo), (whi, wlo) = element_matrices_hp(ops.k)
    with mpmath.workdps(50):
        h = (mpmath.mpf(ops.b) - mpmath.mpf(ops.a)) / (2 * ops.ne)
        h_hi = float(h)
        h_lo = float(h - mpmath.mpf(h_hi))
    q = np.ascontiguousarray(q0, dtype=np.float64)
    lam = np.empty(n)
    s = np.empty((n, n))
    off = 1 if ops.bc == "dirichlet" else 0
    per = 1 if ops.bc == "periodic" else 0
    dp = ctypes.POINTER(ctypes.c_double)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (khi, klo, whi, wlo)]
    st = lib().oracle_eig_jacobi(n, ops.k, ops.ne, off, per, *(a.ctypes.data_as(dp) for a in arrs), h_hi, h_lo,
                                 q.ctypes.data_as(dp), lam.ctypes.data_as(dp), s.ctypes.data_as(dp))
    if st == 1:
        raise MemoryError("oracle_eig_jacobi: allocation failed")
    if st == 2:
        raise RuntimeError("oracle_eig_jacobi: Jacobi sweeps did not converge")
    return lam, s
