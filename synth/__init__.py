"""Seeded synthetic inputs (dense diagonally dominant systems, size and
arrival draws).  Shared by tests and the benchmark; holds none of the Jacobi
method's arithmetic.  The C source ``gen.c`` documents the recipes.

Workload presets (one per measured configuration):

* ``C1``  FP64 n=512, additive margin U[1,2], tol 1e-10, cap 1000
* ``C2``  FP32 n=16384, multiplicative margin U[0.5,1] (a_ii = rowsum*(1+u))
* ``C3``  256 FP32 systems, n log-uniform in [256, 4096], k=32, additive U[1,2]
* ``C4``  FP64 n=32768, multiplicative margin U[0.5,1], stored BF16 for sweeps
* ``C5``  2000 requests, n log-uniform in [256, 16384], k in {1,4,16},
  multiplicative margin U[0.2,1], Poisson arrivals
* ``C4S`` FP64 n=32768 with non-negative off-diagonals U[0,1] (the paper's
  sign pattern) and a_ii = 1.05 rowsum: a slowly converging system
* ``REPLAY`` FP64 systems of the sizes of the paper's serial timing table
  (n = 8 ... 512), additive margin U[1,2]
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gen.c")
LIB = os.path.join(HERE, "libsynth.so")

SEED_BASE = 0x14035805
ADDITIVE = 0
MULTIPLICATIVE = 1
NONNEGATIVE = 2  # off-diagonals U[0,1], multiplicative margin


def seed_for(config_index: int) -> int:
    return SEED_BASE + int(config_index)


def build(out: str = LIB) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-std=c11", "-fPIC", "-shared", SRC, "-o", out + ".tmp",
           "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        build()
    lib = ctypes.CDLL(LIB)
    i64, u64, i32, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.synth_u64.restype = u64
    lib.synth_u64.argtypes = [u64, u64, u64]
    lib.synth_uniform.restype = dbl
    lib.synth_uniform.argtypes = [u64, u64, u64, dbl, dbl]
    lib.synth_dominant.restype = None
    lib.synth_dominant.argtypes = [i64, i64, u64, i32, dbl, dbl, dp, i64, dp, dp]
    lib.synth_dominant_f32.restype = None
    lib.synth_dominant_f32.argtypes = [i64, i64, u64, i32, dbl, dbl, fp, i64, dp, fp]
    lib.synth_paper_uniform.restype = None
    lib.synth_paper_uniform.argtypes = [i64, u64, dp, dp, dp]
    lib.synth_log_uniform_sizes.restype = None
    lib.synth_log_uniform_sizes.argtypes = [i64, u64, i64, i64, ctypes.POINTER(ctypes.c_int64)]
    lib.synth_poisson_arrivals.restype = None
    lib.synth_poisson_arrivals.argtypes = [i64, u64, dbl, dp]
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def dominant(n: int, k: int = 1, seed: int = SEED_BASE, mode: int = ADDITIVE,
             lo: float = 1.0, hi: float = 2.0, lda: int | None = None, out=None):
    """FP64 diagonally dominant system.  Returns (A[n, lda], X_true[n, k], B[n, k]).
    `out` may supply the (n, lda) float64 array for A (e.g. pinned memory)."""
    lib = load()
    lda = lda or n
    A = out if out is not None else np.zeros((n, lda), dtype=np.float64)
    assert A.shape == (n, lda) and A.dtype == np.float64 and A.flags.c_contiguous
    X = np.empty((n, k), dtype=np.float64)
    B = np.empty((n, k), dtype=np.float64)
    lib.synth_dominant(n, k, seed, mode, lo, hi, _dp(A), lda, _dp(X), _dp(B))
    return A, X, B


def dominant_f32(n: int, k: int = 1, seed: int = SEED_BASE, mode: int = ADDITIVE,
                 lo: float = 1.0, hi: float = 2.0, lda: int | None = None):
    """FP32 system of record: (A32[n, lda], X_true[n, k] f64, B32[n, k])."""
    lib = load()
    lda = lda or n
    A = np.zeros((n, lda), dtype=np.float32)
    X = np.empty((n, k), dtype=np.float64)
    B = np.empty((n, k), dtype=np.float32)
    lib.synth_dominant_f32(n, k, seed, mode, lo, hi, _fp(A), lda, _dp(X), _fp(B))
    return A, X, B


def paper_uniform(n: int, seed: int = SEED_BASE):
    """The paper's experiment inputs: A, B, X0 iid U[0,1] (not dominant)."""
    lib = load()
    A = np.empty((n, n), dtype=np.float64)
    B = np.empty(n, dtype=np.float64)
    X0 = np.empty(n, dtype=np.float64)
    lib.synth_paper_uniform(n, seed, _dp(A), _dp(B), _dp(X0))
    return A, B, X0


def log_uniform_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    lib = load()
    out = np.empty(count, dtype=np.int64)
    lib.synth_log_uniform_sizes(count, seed, lo, hi,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return out


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    lib = load()
    out = np.empty(count, dtype=np.float64)
    lib.synth_poisson_arrivals(count, seed, rate, _dp(out))
    return out


def uniform(seed: int, stream: int, count: int, lo: float, hi: float) -> np.ndarray:
    lib = load()
    return np.array([lib.synth_uniform(seed, stream, i, lo, hi) for i in range(count)])


def choice(seed: int, stream: int, count: int, options) -> list:
    """Uniform choice among options for each of count draws."""
    lib = load()
    m = len(options)
    return [options[lib.synth_u64(seed, stream, i) % m] for i in range(count)]


# Presets ------------------------------------------------------------------

def c1():
    """n=512 FP64, additive margin U[1,2]."""
    return dominant(512, 1, seed_for(0), ADDITIVE, 1.0, 2.0)


def c2(n: int = 16384):
    """FP32 n=16384, multiplicative margin U[0.5,1]."""
    return dominant_f32(n, 1, seed_for(1), MULTIPLICATIVE, 0.5, 1.0)


def c3_sizes(count: int = 256):
    return log_uniform_sizes(count, 256, 4096, seed_for(2))


def c3_system(i: int, n: int, k: int = 32):
    """System i of the batched workload (FP32, additive margin U[1,2])."""
    return dominant_f32(n, k, seed_for(2) * 1000003 + i, ADDITIVE, 1.0, 2.0)


def c4(n: int = 32768):
    """FP64 n=32768, multiplicative margin U[0.5,1] (swept in BF16)."""
    return dominant(n, 1, seed_for(3), MULTIPLICATIVE, 0.5, 1.0)


def c4_slow(n: int = 32768):
    """FP64 n=32768, off-diagonals U[0,1], a_ii = 1.05 rowsum (spectral radius
    of the Jacobi matrix 1/1.05)."""
    return dominant(n, 1, seed_for(5), NONNEGATIVE, 0.05, 0.05)


REPLAY_SIZES = (8, 16, 32, 64, 128, 256, 512)


def replay_system(n: int):
    """FP64 system of one size of the paper's serial timing table."""
    return dominant(n, 1, seed_for(6) * 1000003 + n, ADDITIVE, 1.0, 2.0)


C5_STREAM_K = 9
C5_STREAM_DTYPE = 10


def c5_requests(count: int = 2000):
    """Serving workload: per request (n, k, sweep dtype); n log-uniform in
    [256, 16384], k uniform over {1, 4, 16}, FP32 or BF16 inner sweeps 50/50."""
    sd = seed_for(4)
    ns = log_uniform_sizes(count, 256, 16384, sd)
    ks = choice(sd, C5_STREAM_K, count, [1, 4, 16])
    dts = choice(sd, C5_STREAM_DTYPE, count, ["f32", "bf16"])
    return [(int(n), int(k), d) for n, k, d in zip(ns, ks, dts)]


def c5_system(i: int, n: int, k: int, out=None):
    """System for request i: multiplicative margin U[0.2,1]."""
    return dominant(n, k, seed_for(4) * 1000003 + i, MULTIPLICATIVE, 0.2, 1.0, out=out)
