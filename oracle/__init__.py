"""Serial FP64 CPU oracle for the Jacobi iteration (ctypes binding).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library and its Python
binding never do.  The C source (``jacobi_oracle.c``) follows sec. 2 of the
paper (component equation and serial pseudocode); see its header for the
readings taken where the paper is silent or garbled.

``build()`` compiles ``libjacobi_oracle.so`` with gcc.  ``load()`` returns the
built library, compiling it only when none exists.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "jacobi_oracle.c")
LIB = os.path.join(HERE, "libjacobi_oracle.so")

# Status codes of the oracle (same numeric values as the library's).
OK = 0
NOT_CONVERGED = 1
DIVERGED = 2
ERR_INVALID_ARG = -1
ERR_ZERO_DIAGONAL = -2
ERR_NONFINITE_INPUT = -3
ERR_OUT_OF_MEMORY = -4

NORM_INF = 0
NORM_L2 = 1


class OracleInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("bad_index", ctypes.c_int64),
        ("final_delta", ctypes.c_double),
    ]


def build(src: str = SRC, out: str = LIB, extra: list[str] | None = None) -> str:
    """Compile the oracle.  -ffp-contract=off keeps multiply and add separate."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC",
           "-shared", src, "-o", out + ".tmp", "-lm"] + (extra or [])
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_lib = None


def load(path: str = LIB):
    global _lib
    if path == LIB and _lib is not None:
        return _lib
    if not os.path.exists(path):
        build(out=path)
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    i64 = ctypes.c_int64
    lib.oracle_jacobi.restype = ctypes.c_int32
    lib.oracle_jacobi.argtypes = [i64, i64, dp, i64, dp, i64, dp, dp, i64, ctypes.c_double,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(OracleInfo)]
    lib.oracle_update_rows.restype = None
    lib.oracle_update_rows.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64,
                                       ctypes.POINTER(ctypes.c_int64), i64, dp]
    lib.oracle_update_rows_f32.restype = None
    lib.oracle_update_rows_f32.argtypes = [i64, i64, fp, i64, dp, i64, dp, i64,
                                           ctypes.POINTER(ctypes.c_int64), i64, dp]
    lib.oracle_residual.restype = None
    lib.oracle_residual.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64, dp, i64]
    lib.oracle_round_bf16.restype = ctypes.c_double
    lib.oracle_round_bf16.argtypes = [ctypes.c_double]
    lib.oracle_round_bf16_array.restype = None
    lib.oracle_round_bf16_array.argtypes = [dp, dp, i64]
    if path == LIB:
        _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as2d(a, k_hint=None) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    return np.ascontiguousarray(a)


def jacobi(A, B, X0=None, tol=1e-8, max_iter=10000, norm="inf", lib=None):
    """Run the oracle.  A (n x n), B (n x k or n), X0 like B or None.

    Returns (X, info) with X shaped like B and info a dict with status,
    iterations, bad_index, final_delta.
    """
    lib = lib or load()
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    vec = np.asarray(B).ndim == 1
    B2 = _as2d(B)
    n, k = B2.shape
    if A.shape[0] != n:
        raise ValueError("A and B disagree on n")
    X0p = None
    if X0 is not None:
        X0a = _as2d(X0)
        X0p = _dptr(X0a)
    X = np.zeros((n, k), dtype=np.float64)
    info = OracleInfo()
    nrm = NORM_L2 if norm in ("l2", NORM_L2) else NORM_INF
    lib.oracle_jacobi(n, k, _dptr(A), A.shape[1], _dptr(B2), k, X0p, _dptr(X), k,
                      float(tol), int(max_iter), nrm, ctypes.byref(info))
    out = X[:, 0].copy() if vec else X
    return out, dict(status=info.status, iterations=info.iterations,
                     bad_index=info.bad_index, final_delta=info.final_delta)


def update_rows(A, B, Xold, rows, lib=None):
    """One Jacobi update at the given rows from Xold (component equation).

    A may be float64 or float32 (the promoted FP32 system); B and Xold are
    promoted to float64.  Returns an array (len(rows), k)."""
    lib = lib or load()
    B2 = _as2d(B)
    Xo = _as2d(Xold)
    n, k = B2.shape
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    out = np.zeros((rows.size, k), dtype=np.float64)
    rp = rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    if A.dtype == np.float32:
        A = np.ascontiguousarray(A)
        lib.oracle_update_rows_f32(n, k, A.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                   A.shape[1], _dptr(B2), k, _dptr(Xo), k, rp, rows.size,
                                   _dptr(out))
    else:
        A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
        lib.oracle_update_rows(n, k, _dptr(A), A.shape[1], _dptr(B2), k, _dptr(Xo), k, rp,
                               rows.size, _dptr(out))
    return out


def residual(A, B, X, lib=None):
    """R = B - A X in plain FP64."""
    lib = lib or load()
    A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    vec = np.asarray(B).ndim == 1
    B2 = _as2d(B)
    X2 = _as2d(X)
    n, k = B2.shape
    R = np.zeros((n, k), dtype=np.float64)
    lib.oracle_residual(n, k, _dptr(A), A.shape[1], _dptr(B2), k, _dptr(X2), k, _dptr(R), k)
    return R[:, 0].copy() if vec else R


def round_bf16(x, lib=None) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even), as float64."""
    lib = lib or load()
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    out = np.empty_like(a)
    lib.oracle_round_bf16_array(_dptr(a), _dptr(out), a.size)
    return out
