"""Python access to the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the product package.  It shares no code
with the HIP library; both sides meet only through the seeded inputs of
paper_2501_02483_amd/inputs.py.

All functions use the row-profile ("skyline") layout: row i stores columns
f[i]..i contiguously; arrow rows have f == 0.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)


def build(force=True):
    """Compile oracle.c with gcc -O2 (no fast-math) and OpenMP."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_factor.restype = ctypes.c_int64
        lib.oracle_factor.argtypes = [ctypes.c_int64, _i64p, _f64p, ctypes.c_int]
        lib.oracle_logdet.restype = ctypes.c_double
        lib.oracle_logdet.argtypes = [ctypes.c_int64, _i64p, _f64p]
        lib.oracle_solve.restype = None
        lib.oracle_solve.argtypes = [ctypes.c_int64, _i64p, _f64p, ctypes.c_int64, _f64p, ctypes.c_int64]
        lib.oracle_symv.restype = None
        lib.oracle_symv.argtypes = [ctypes.c_int64, _i64p, _f64p, ctypes.c_int64, _f64p,
                                    ctypes.c_int64, _f64p, ctypes.c_int64]
        lib.oracle_factor_residual.restype = None
        lib.oracle_factor_residual.argtypes = [ctypes.c_int64, _i64p, _f64p, _f64p, ctypes.c_int64,
                                               _i64p, _f64p, _f64p]
        lib.oracle_selinv.restype = None
        lib.oracle_selinv.argtypes = [ctypes.c_int64, _i64p, _f64p, _f64p, ctypes.c_int]
        lib.oracle_row_ptr.restype = None
        lib.oracle_row_ptr.argtypes = [ctypes.c_int64, _i64p, _i64p]
        _lib = lib
    return _lib


def _p64(a):
    return a.ctypes.data_as(_f64p)


def _pi(a):
    return a.ctypes.data_as(_i64p)


def _prof(f):
    f = np.ascontiguousarray(f, dtype=np.int64)
    return f


def row_ptr(f):
    f = _prof(f)
    rp = np.empty(f.shape[0] + 1, dtype=np.int64)
    _load().oracle_row_ptr(f.shape[0], _pi(f), _pi(rp))
    return rp


def factor(f, values, nthreads=0):
    """Envelope Cholesky. Returns (L values in the same layout, info)."""
    f = _prof(f)
    L = np.array(values, dtype=np.float64, copy=True)
    info = _load().oracle_factor(f.shape[0], _pi(f), _p64(L), int(nthreads))
    return L, int(info)


def logdet(f, L):
    f = _prof(f)
    L = np.ascontiguousarray(L, dtype=np.float64)
    return float(_load().oracle_logdet(f.shape[0], _pi(f), _p64(L)))


def solve(f, L, B):
    """X = A^{-1} B with A = L L^T; B is (N,) or (N, nrhs)."""
    f = _prof(f)
    L = np.ascontiguousarray(L, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    vec = B.ndim == 1
    X = np.array(B.reshape(B.shape[0], -1), dtype=np.float64, order="F", copy=True)
    _load().oracle_solve(f.shape[0], _pi(f), _p64(L), X.shape[1], _p64(X), X.shape[0])
    return X[:, 0].copy() if vec else X


def selinv(f, L, nthreads=0):
    """Entries of A^{-1} inside the envelope, from the factor L (same layout)."""
    f = _prof(f)
    L = np.ascontiguousarray(L, dtype=np.float64)
    Sg = np.zeros_like(L)
    _load().oracle_selinv(f.shape[0], _pi(f), _p64(L), _p64(Sg), int(nthreads))
    return Sg


def symv(f, A, X):
    """Y = A X for the symmetric matrix given by its lower envelope."""
    f = _prof(f)
    A = np.ascontiguousarray(A, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    vec = X.ndim == 1
    Xf = np.array(X.reshape(X.shape[0], -1), dtype=np.float64, order="F", copy=True)
    Y = np.zeros_like(Xf, order="F")
    _load().oracle_symv(f.shape[0], _pi(f), _p64(A), Xf.shape[1], _p64(Xf), Xf.shape[0],
                        _p64(Y), Y.shape[0])
    return Y[:, 0].copy() if vec else Y


def factor_residual(f, A, L, rows=None):
    """||L L^T - A||_F / ||A||_F restricted to the given rows (all rows if None)."""
    f = _prof(f)
    if rows is None:
        rows = np.arange(f.shape[0], dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    num = ctypes.c_double()
    den = ctypes.c_double()
    _load().oracle_factor_residual(f.shape[0], _pi(f), _p64(np.ascontiguousarray(A, dtype=np.float64)),
                                   _p64(np.ascontiguousarray(L, dtype=np.float64)), rows.shape[0],
                                   _pi(rows), ctypes.byref(num), ctypes.byref(den))
    return float(np.sqrt(num.value / den.value))
