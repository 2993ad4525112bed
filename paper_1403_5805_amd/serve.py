"""Serving: continuous-batching solve server (jacobi_serve_*).  Argument
marshalling only; requests are host (numpy) FP64 arrays kept alive here
until their ticket completes."""
from __future__ import annotations

import ctypes
import threading

import numpy as np

from . import _lib


class Server:
    """A solve server on one device.

        srv = Server(max_active=64)
        t = srv.submit(A, B, sweep_dtype="bf16", rel_tol=1e-12)   # numpy float64
        X, info = srv.wait(t)
        srv.stats(); srv.close()
    """

    def __init__(self, device: int = 0, max_active: int = 64, hbm_budget_bytes: int = 0,
                 inner_max: int = 64, max_outer: int = 50, inner_rel_tol: float = 1e-3):
        lib = _lib.load()
        cfg = _lib.ServeConfig()
        lib.jacobi_serve_config_default(ctypes.byref(cfg))
        cfg.device = device
        cfg.max_active = max_active
        cfg.hbm_budget_bytes = hbm_budget_bytes
        cfg.inner_max = inner_max
        cfg.max_outer = max_outer
        cfg.inner_rel_tol = inner_rel_tol
        h = ctypes.c_void_p()
        st = lib.jacobi_serve_create(ctypes.byref(cfg), ctypes.byref(h))
        if st != 0:
            raise RuntimeError(f"jacobi_serve_create failed: {st}: "
                               f"{lib.jacobi_last_error().decode()}")
        self._lib = lib
        self.handle = h
        self._keep = {}
        self._mu = threading.Lock()
        _lib.track(self)

    def submit(self, A: np.ndarray, B: np.ndarray, out: np.ndarray | None = None,
               sweep_dtype: str = "bf16", rel_tol: float = 1e-12, max_outer: int = 0):
        """Queue A x = B (host float64 arrays, B (n,) or (n, k)).  max_outer caps
        this request's refinement steps (0: the server's cap).  Returns
        (ticket, status) where status is 0 when queued, else the error code."""
        A = np.ascontiguousarray(A, dtype=np.float64)
        if B.ndim not in (1, 2):
            raise ValueError("B must be (n,) or (n, k)")
        vec = B.ndim == 1
        B2 = np.ascontiguousarray(B.reshape(B.shape[0], -1), dtype=np.float64)
        n, k = B2.shape
        if A.ndim != 2 or A.shape != (n, n):
            raise ValueError(f"A must be ({n}, {n}) (got {A.shape})")
        if out is not None:
            if (out.dtype != np.float64 or not out.flags.c_contiguous or
                    out.size != n * k or out.shape[0] != n):
                raise ValueError("out must be a C-contiguous float64 array shaped like B")
        X = out if out is not None else np.zeros((n, k), dtype=np.float64)
        req = _lib.Request()
        req.n, req.k = n, k
        req.A, req.lda = A.ctypes.data, A.shape[1]
        req.B, req.ldb = B2.ctypes.data, k
        req.X, req.ldx = X.ctypes.data, k
        req.sweep_dtype = {"f32": 1, "bf16": 2}[sweep_dtype]
        req.rel_tol = rel_tol
        req.max_outer = int(max_outer)
        t = ctypes.c_uint64()
        st = self._lib.jacobi_serve_submit(self.handle, ctypes.byref(req), ctypes.byref(t))
        with self._mu:
            self._keep[t.value] = (A, B2, X, vec)
        return t.value, st

    def _result(self, t, info):
        with self._mu:
            A, B2, X, vec = self._keep.get(t, (None, None, None, False))
        d = info.as_dict()
        return (X[:, 0] if (vec and X is not None and X.ndim == 2) else X), d

    def poll(self, t):
        info = _lib.Info()
        self._lib.jacobi_serve_poll(self.handle, t, ctypes.byref(info))
        return self._result(t, info)

    def wait(self, t, timeout_s: float | None = None):
        info = _lib.Info()
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        self._lib.jacobi_serve_wait(self.handle, t, us, ctypes.byref(info))
        X, d = self._result(t, info)
        if d["status"] != 3:  # not PENDING: release the host arrays
            with self._mu:
                self._keep.pop(t, None)
        return X, d

    def stats(self) -> dict:
        st = _lib.ServeStats()
        self._lib.jacobi_serve_stats_get(self.handle, ctypes.byref(st))
        return st.as_dict()

    def close(self):
        if self.handle:
            self._lib.jacobi_serve_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
