"""Python entry to the C cyclic-Jacobi oracle (see jacobi.c).

Oracle code: test infrastructure only.  The shared library is compiled with
gcc from ``jacobi.c`` next to this file; nothing here touches the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jacobi.c")
_LIB = os.path.join(_HERE, "_oracle_jacobi.so")
_lib = None


def build_jacobi_lib(force: bool = False) -> str:
    """Compile jacobi.c with gcc (plain -O2, no fast-math so IEEE rounding holds)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build_jacobi_lib()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_jacobi_eigh.restype = ctypes.c_int
        lib.oracle_jacobi_eigh.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_void_p, ctypes.c_int64, ctypes.c_double,
                                           ctypes.c_int]
        _lib = lib
    return _lib


def jacobi_eigh(A: np.ndarray, tol: float = 2.0 ** -53, max_sweeps: int = 100):
    """Eigen-decomposition of a real symmetric matrix by cyclic Jacobi.

    Returns (lam, U, sweeps) with lam ascending (stable order among ties) and
    U's columns the matching orthonormal eigenvectors, so A = U diag(lam) U^T
    (Eq. 3).  A is not modified.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    assert A.shape == (n, n)
    a = np.array(A, dtype=np.float64, order="F", copy=True)
    v = np.zeros((n, n), dtype=np.float64, order="F")
    if n == 0:
        return np.zeros(0), v, 0
    sweeps = _load().oracle_jacobi_eigh(n, a.ctypes.data, n, v.ctypes.data, n, float(tol), int(max_sweeps))
    if sweeps < 0:
        raise RuntimeError("Jacobi did not converge in %d sweeps" % max_sweeps)
    lam = np.diag(a).copy()
    order = np.argsort(lam, kind="stable")
    return lam[order], np.ascontiguousarray(v[:, order]), sweeps
