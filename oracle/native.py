"""ctypes loader of ``dirac_sites.c``: the oracle's operator written out in
plain C (FP64, OpenMP over sites) for whole-lattice residual checks at sizes
where ``dirac.py`` is too slow.

TEST INFRASTRUCTURE ONLY (see the package docstring).  ``build()`` compiles
the shared library next to its source with gcc; ``lib()`` loads it, building
it first if it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dirac_sites.c")
LIB = os.path.join(HERE, "liboracle_dirac.so")

_lib = None


def build() -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fcx-limited-range", "-fPIC", "-shared", SRC, "-o", tmp, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"oracle C build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        l = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        l.oracle_local_matrix.argtypes = [ip, dp, ctypes.c_double, ctypes.c_double, dp]
        l.oracle_apply.argtypes = [ip, dp, dp, ctypes.c_double, ctypes.c_int, dp, dp, ctypes.c_int]
        l.oracle_residual.argtypes = [ip, dp, dp, ctypes.c_double, ctypes.c_int, dp, dp, ctypes.c_int, dp, dp]
        for f in (l.oracle_local_matrix, l.oracle_apply, l.oracle_residual):
            f.restype = ctypes.c_int
        _lib = l
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.complex128 or a.dtype == np.float64
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _dims(U: np.ndarray):
    lt, lz, ly, lx = U.shape[1:5]
    return (ctypes.c_int * 4)(lx, ly, lz, lt)


def local_matrix(U: np.ndarray, kappa: float, csw: float) -> np.ndarray:
    """The 12x12 site-local matrix of Eq. (1) per site, shape (V, 12, 12)."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    V = int(np.prod(U.shape[1:5]))
    M = np.empty((V, 12, 12), dtype=np.complex128)
    assert lib().oracle_local_matrix(_dims(U), _dp(U), kappa, csw, _dp(M)) == 0
    return M


def apply(U: np.ndarray, kappa: float, M: np.ndarray, X: np.ndarray, dagger: bool = False) -> np.ndarray:
    """D_W X (or D_W^dagger X) with a precomputed ``local_matrix``; X of
    shape (..., 4, 3, L) over the lattice in the oracle's layout."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    X = np.ascontiguousarray(X, dtype=np.complex128)
    L = X.shape[-1]
    Y = np.empty_like(X)
    assert lib().oracle_apply(_dims(U), _dp(U), _dp(M), kappa, L, _dp(X), _dp(Y), int(dagger)) == 0
    return Y


def residual(U: np.ndarray, kappa: float, M: np.ndarray, X: np.ndarray, B: np.ndarray, dagger: bool = False):
    """Per column: ||b_i - D x_i|| / ||b_i|| over the whole lattice (the true
    residual of Sec. 4.3), and ||b_i||."""
    U = np.ascontiguousarray(U, dtype=np.complex128)
    X = np.ascontiguousarray(X, dtype=np.complex128)
    B = np.ascontiguousarray(B, dtype=np.complex128)
    assert X.shape == B.shape
    L = X.shape[-1]
    r2 = np.zeros(L)
    b2 = np.zeros(L)
    assert lib().oracle_residual(_dims(U), _dp(U), _dp(M), kappa, L, _dp(X), _dp(B), int(dagger), _dp(r2), _dp(b2)) == 0
    return np.sqrt(r2) / np.sqrt(b2), np.sqrt(b2)
