"""MI355X (gfx950) dense Jacobi solver: Python binding of libjacobi.

The method is the Jacobi iteration for A X = B of Margaris, Souravlas and
Roumeliotis (sec. 2: component equation and serial pseudocode).  Every step
runs in the library's HIP kernels; this module only marshals torch device
tensors and the current torch stream into the C ABI (include/jacobi.h).

    import torch, paper_1403_5805_amd as jac
    X, info = jac.solve(A, B, tol=1e-8, max_iter=10000)

Defaults tol = 1e-8 and max_iter = 10000 are the paper's experiment values
(sec. 4).
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (BF16, CANCELLED, DIVERGED, ERR_DEVICE, ERR_INTERNAL, ERR_INVALID_ARG,
                   ERR_NONFINITE_INPUT, ERR_OUT_OF_MEMORY, ERR_REJECTED, ERR_ZERO_DIAGONAL, F32,
                   F64, NOT_CONVERGED, OK, PENDING, Info, Options)

__all__ = ["solve", "solve_noalloc", "stream_probe", "solve_batched", "Batch", "Server",
           "Matrix", "status_string", "last_error", "Context",
           "OK", "NOT_CONVERGED", "DIVERGED", "PENDING", "CANCELLED", "ERR_INVALID_ARG",
           "ERR_ZERO_DIAGONAL", "ERR_NONFINITE_INPUT", "ERR_OUT_OF_MEMORY", "ERR_DEVICE",
           "ERR_REJECTED", "ERR_INTERNAL", "F64", "F32", "BF16"]


def _torch():
    import torch
    return torch


_STATUS_NAMES: dict = {}


def status_string(code: int) -> str:
    code = int(code)
    name = _STATUS_NAMES.get(code)
    if name is None:
        name = _STATUS_NAMES[code] = _lib.load().jacobi_status_string(code).decode()
    return name


def last_error() -> str:
    return _lib.load().jacobi_last_error().decode()


def _a_dtype(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    raise TypeError(f"unsupported dtype for A: {t.dtype}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _ld(t) -> int:
    """Leading dimension of a row-major 2-D view (unit column stride)."""
    if t.dim() == 1:
        if t.stride(0) != 1:
            raise ValueError("vectors must be contiguous")
        return 1
    if t.stride(1) != 1:
        raise ValueError("matrices must have unit column stride (row-major)")
    return max(t.stride(0), t.shape[1])


def _vec_dtype(a_dtype: int, mode: str = "plain"):
    """Element type of B, x0 and X for a given A type (include/jacobi.h)."""
    torch = _torch()
    return torch.float64 if (a_dtype == F64 or mode in ("refine", 1)) else torch.float32


def _check_operand(t, name: str, device, dtype, shape) -> int:
    """Reject what would make the library read or write outside a tensor:
    host tensors, another device, another element type or shape, and row
    views whose rows overlap (row stride below the row length).  Returns the
    leading dimension (1 for a vector)."""
    if t.is_cuda and t.device == device and t.dtype == dtype and t.shape == shape:
        st = t.stride()
        if len(st) == 1 and st[0] == 1:
            return 1
        if len(st) == 2 and st[1] == 1 and (shape[0] <= 1 or st[0] >= shape[1]):
            return max(st[0], shape[1])
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (got device {t.device})")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, A is on {device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    if t.dim() == 2 and t.shape[0] > 1 and t.stride(0) < t.shape[1]:
        raise ValueError(f"{name}: rows overlap (row stride {t.stride(0)} < {t.shape[1]})")
    return _ld(t)


def make_options(tol=1e-8, max_iter=10000, norm="inf", mode="plain", sweep_dtype="bf16",
                 inner_rel_tol=1e-3, max_inner=200, max_outer=50, refine_tol=1e-12,
                 sync_every=0, profile=False) -> Options:
    o = Options()
    _lib.load().jacobi_options_default(ctypes.byref(o))
    o.tol = float(tol)
    o.max_iter = int(max_iter)
    o.norm = {"inf": 0, "l2": 1}[norm] if isinstance(norm, str) else int(norm)
    o.mode = {"plain": 0, "refine": 1}[mode] if isinstance(mode, str) else int(mode)
    o.sweep_dtype = ({"f32": F32, "bf16": BF16}[sweep_dtype]
                     if isinstance(sweep_dtype, str) else int(sweep_dtype))
    o.inner_rel_tol = float(inner_rel_tol)
    o.max_inner = int(max_inner)
    o.max_outer = int(max_outer)
    o.refine_tol = float(refine_tol)
    o.sync_every = int(sync_every)
    o.profile = 1 if profile else 0
    return o


_OPTIONS_CACHE: dict = {}


def _options(opts: dict) -> Options:
    """make_options(**opts), kept per distinct keyword set (the library reads
    the struct through a const pointer and never changes it)."""
    try:
        key = tuple(sorted(opts.items()))
        o = _OPTIONS_CACHE.get(key)
    except TypeError:  # an unhashable value: build it every time
        return make_options(**opts)
    if o is None:
        o = make_options(**opts)
        if len(_OPTIONS_CACHE) >= 256:
            _OPTIONS_CACHE.clear()
        _OPTIONS_CACHE[key] = o
    return o


class Context:
    """A solver context bound to one device (owns reusable workspaces)."""

    def __init__(self, device: int = 0):
        lib = _lib.load()
        h = ctypes.c_void_p()
        st = lib.jacobi_ctx_create(int(device), ctypes.byref(h))
        if st != OK:
            raise RuntimeError(f"jacobi_ctx_create: {status_string(st)} {last_error()}")
        self.handle = h
        _lib.track(self)

    def close(self):
        if self.handle:
            _lib.load().jacobi_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_handle(stream, device):
    torch = _torch()
    if stream is not None:
        return ctypes.c_void_p(stream.cuda_stream)
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:  # the current stream's handle without a Stream object
        idx = device.index if getattr(device, "index", None) is not None else \
            torch.cuda.current_device()
        return ctypes.c_void_p(raw(idx))
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def solve(A, B, x0=None, *, out=None, ctx: Context | None = None, stream=None,
          raise_on_error: bool = False, _noalloc: bool = False, _matrix=None, **opts):
    """Solve A X = B by Jacobi sweeps on the GPU.

    A: (n, n) torch tensor on the GPU, float64 / float32 / bfloat16, unit column
    stride (a row stride > n is honoured as the leading dimension).
    B: (n,) or (n, k); float64 for float64 A (and in refine mode), else float32.
    x0: initial approximation like B, or None for zero.
    opts: tol, max_iter, norm ("inf" | "l2"), mode ("plain" | "refine"),
    sweep_dtype ("f32" | "bf16"), inner_rel_tol, max_inner, max_outer,
    refine_tol, sync_every, profile.
    Returns (X, info dict).  X has B's shape.
    """
    torch = _torch()
    lib = _lib.load()
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    n = A.shape[0]
    vec = B.dim() == 1
    k = 1 if vec else B.shape[1]
    if B.shape[0] != n or B.dim() > 2:
        raise ValueError("B must be (n,) or (n, k)")
    dt = _a_dtype(A)
    lda = _check_operand(A, "A", A.device, A.dtype, (n, n))
    vdt = _vec_dtype(dt, opts.get("mode", "plain"))
    ldb = _check_operand(B, "B", A.device, vdt, B.shape)
    if out is None:
        out = torch.empty((n,) if vec else (n, k), dtype=B.dtype, device=B.device)
    ldx = _check_operand(out, "out", A.device, vdt, B.shape)
    if x0 is not None:
        ld0 = _check_operand(x0, "x0", A.device, vdt, B.shape)
        if not vec and ld0 != ldx:
            # X0 is read with out's leading dimension
            x0 = torch.empty((n, ldx), dtype=vdt, device=A.device)[:, :k].copy_(x0)
    noalloc = _noalloc
    o = _options(opts)
    info = Info()
    args = (n, k, dt, _ptr(A), lda, _ptr(B), ldb, _ptr(x0) if x0 is not None else None,
            _ptr(out), ldx, ctypes.byref(o), _stream_handle(stream, A.device),
            ctypes.byref(info))
    if noalloc:
        if ctx is not None:
            raise ValueError("the no-allocation entry point takes no context")
        st = lib.jacobi_solve_noalloc(*args)
    elif _matrix is not None:
        st = lib.jacobi_solve_prepared(_matrix.handle, *args[1:2], *args[5:])
    else:
        st = lib.jacobi_solve(ctx.handle if ctx else None, *args)
    d = info.as_dict()
    d["status_name"] = status_string(st)
    if st < 0:
        d["error"] = last_error()
        if raise_on_error:
            raise RuntimeError(f"jacobi_solve failed: {d['status_name']}: {d['error']}")
    return out, d


def stream_probe(buf, *, reps: int = 5, stream=None) -> dict:
    """jacobi_stream_probe: the achievable HBM read rate over a device tensor
    (read only; at least 16 bytes; larger than the caches for the HBM rate).
    Returns {"GBps": fastest rate, "wg_per_cu": its launch shape}."""
    lib = _lib.load()
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("stream_probe needs a contiguous device tensor")
    g = ctypes.c_double()
    w = ctypes.c_int32()
    st = lib.jacobi_stream_probe(_ptr(buf), buf.numel() * buf.element_size(), int(reps),
                                 _stream_handle(stream, buf.device), ctypes.byref(g),
                                 ctypes.byref(w))
    if st != OK:
        raise RuntimeError(f"jacobi_stream_probe: {status_string(st)} {last_error()}")
    return {"GBps": g.value, "wg_per_cu": w.value}


def solve_noalloc(A, B, x0=None, *, out=None, stream=None, raise_on_error: bool = False,
                  **opts):
    """jacobi_solve_noalloc: the plain solve with its workspace in the
    library's fixed per-device array (no device allocation by the library;
    k <= 2, plain mode).  The caller provides `out` to avoid torch allocating
    the result.  Same arguments and results as solve()."""
    return solve(A, B, x0, out=out, stream=stream, raise_on_error=raise_on_error,
                 _noalloc=True, **opts)


class Matrix:
    """A prepared matrix (jacobi_matrix_create): A kept for repeated solves
    with new right-hand sides.  With sweep_dtype ("f32" | "bf16"; float64 A
    only) the reduced-precision copy that refinement sweeps is built once, here,
    instead of on every refine solve.  A must not change while the Matrix is
    open.  solve() takes solve()'s arguments and gives the same results."""

    def __init__(self, A, *, sweep_dtype: str | None = None, ctx: Context | None = None,
                 stream=None):
        lib = _lib.load()
        if A.dim() != 2 or A.shape[0] != A.shape[1]:
            raise ValueError("A must be square")
        n = A.shape[0]
        dt = _a_dtype(A)
        _check_operand(A, "A", A.device, A.dtype, (n, n))
        lo = -1 if sweep_dtype is None else {"f32": F32, "bf16": BF16}[sweep_dtype]
        h = ctypes.c_void_p()
        st = lib.jacobi_matrix_create(ctx.handle if ctx else None, n, dt, _ptr(A), _ld(A), lo,
                                      _stream_handle(stream, A.device), ctypes.byref(h))
        if st != OK:
            raise RuntimeError(f"jacobi_matrix_create: {status_string(st)} {last_error()}")
        self.A, self.ctx, self.handle = A, ctx, h
        _lib.track(self)

    def solve(self, B, x0=None, *, out=None, stream=None, raise_on_error: bool = False,
              **opts):
        if not self.handle:
            raise RuntimeError("the matrix is closed")
        return solve(self.A, B, x0, out=out, ctx=self.ctx, stream=stream,
                     raise_on_error=raise_on_error, _matrix=self, **opts)

    def close(self):
        if self.handle:
            _lib.load().jacobi_matrix_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


from .batched import Batch, solve_batched  # noqa: E402
from .serve import Server  # noqa: E402
