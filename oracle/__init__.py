"""CPU oracle for the rank-k Cholesky modification (test infrastructure).

This package is TEST INFRASTRUCTURE.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path
(the HIP library and its binding) never does, and the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, FP64, compiled without FMA
contraction or fast-math); this module only builds it with gcc and marshals
numpy arrays through ctypes.  Each wrapper names the part of the paper
(Walder 2010, "Rank k Cholesky Up/Down-dating on the GPU") it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, ARG, NOT_PD, BAD_DIAG = 0, -1, -2, -3

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, no FP contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fno-unsafe-math-optimizations", "-Wall", "-shared", "-fPIC",
           _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        ci = ctypes.c_int
        lib.oracle_modify.argtypes = [p, p, i64, i64, i64, ci, p, p]
        lib.oracle_modify_seq.argtypes = [p, p, i64, i64, i64, ci, p, p]
        lib.oracle_modify_colA.argtypes = [p, p, i64, i64, i64, ci, p]
        lib.oracle_cholesky_upper.argtypes = [p, i64, p, i64, i64, p]
        lib.oracle_target_matrix.argtypes = [p, i64, p, i64, i64, ci, p]
        for f in (lib.oracle_modify, lib.oracle_modify_seq, lib.oracle_modify_colA,
                  lib.oracle_cholesky_upper, lib.oracle_target_matrix):
            f.restype = ci
        _lib = lib
        return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _as_L(L):
    L = np.ascontiguousarray(L, dtype=np.float64)
    if L.ndim != 2 or L.shape[1] < L.shape[0]:
        raise ValueError("L must be (n, ldl) with ldl >= n")
    return L


def _as_V(V, n):
    V = np.asarray(V, dtype=np.float64)
    if V.ndim == 1:
        V = V.reshape(n, 1)
    V = np.ascontiguousarray(V)
    if V.shape[0] != n:
        raise ValueError("V must have n rows")
    return V


class OracleError(RuntimeError):
    def __init__(self, status, info, k):
        self.status, self.info = status, info
        self.row, self.col = (info // k, info % k) if (info >= 0 and k > 0) else (-1, -1)
        super().__init__("oracle status %d at (row %d, col %d)" % (status, self.row, self.col))


def modify(L, V, sigma, *, seq=False, return_w=False, raise_on_error=False):
    """Rank-k CholeskyModifyB (Algorithm 1, second alternative), serial FP64.

    Returns (L_new, status, info[, W]); L is not modified.  ``seq=True`` runs
    k literal rank-1 passes instead of the row-interleaved rank-k loop.
    """
    L = _as_L(L).copy()
    n, ldl = L.shape
    V = _as_V(V, n)
    k = V.shape[1]
    W = np.empty((n, k), dtype=np.float64) if return_w else None
    info = ctypes.c_int64(-1)
    fn = _load().oracle_modify_seq if seq else _load().oracle_modify
    st = fn(_ptr(L), _ptr(V), n, k, ldl, int(sigma), _ptr(W), ctypes.byref(info))
    if raise_on_error and st != OK:
        raise OracleError(st, info.value, k)
    return (L, st, info.value, W) if return_w else (L, st, info.value)


def modify_colA(L, V, sigma):
    """Corrected CholeskyModifyA (Algorithm 1, first alternative), FP64."""
    L = _as_L(L).copy()
    n, ldl = L.shape
    V = _as_V(V, n)
    info = ctypes.c_int64(-1)
    st = _load().oracle_modify_colA(_ptr(L), _ptr(V), n, V.shape[1], ldl, int(sigma),
                                    ctypes.byref(info))
    return L, st, info.value


def cholesky_upper(A):
    """Textbook upper Cholesky A = U^T U (FP64); raises on a non-positive pivot."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    U = np.zeros((n, n), dtype=np.float64)
    info = ctypes.c_int64(-1)
    st = _load().oracle_cholesky_upper(_ptr(A), max(n, 1), _ptr(U), max(n, 1), n,
                                       ctypes.byref(info))
    if st != OK:
        raise OracleError(st, info.value, 1)
    return U


def target_matrix(L, V, sigma):
    """A~ = L^T L + sigma V V^T (Section 1), dense FP64, O(n^3)."""
    L = _as_L(L)
    n, ldl = L.shape
    V = _as_V(V, n)
    At = np.empty((n, n), dtype=np.float64)
    st = _load().oracle_target_matrix(_ptr(L), ldl, _ptr(V), n, V.shape[1], int(sigma), _ptr(At))
    if st != OK:
        raise OracleError(st, -1, 1)
    return At
