"""Batched solves: many independent systems in one persistent launch
(jacobi_solve_batched).  Argument marshalling only."""
from __future__ import annotations

import ctypes

from . import _lib


class Batch:
    """A batch of systems marshalled once for repeated solves.

    `systems` holds (A, B) or (A, B, x0) tuples as for solve_batched; the
    operands are checked and their pointers, sizes and leading dimensions
    packed into the C array here, once.  Every solve() call then solves all
    systems from their x0 (or zero) with the options given, writing the
    outputs `xs`.  The tensors must stay alive and keep their storage while
    the Batch is used (their contents may change between solves)."""

    def __init__(self, systems, *, outs=None, ctx=None):
        import torch

        from . import _a_dtype, _check_operand, _vec_dtype
        self._lib = _lib.load()
        self.ctx = ctx
        self.count = count = len(systems)
        self.xs = []
        self._keep = []
        if count == 0:
            return
        self.dtype = dt = _a_dtype(systems[0][0])
        self.device = dev = systems[0][0].device
        self._arr = arr = (_lib.System * count)()
        adt = systems[0][0].dtype
        vdt = _vec_dtype(dt)
        for i, sysd in enumerate(systems):
            A, B = sysd[0], sysd[1]
            x0 = sysd[2] if len(sysd) > 2 else None
            if A.dtype != adt:
                raise TypeError("all systems of a batch share A's dtype")
            bshape = B.shape
            vec = len(bshape) == 1
            n = A.shape[0]
            k = 1 if vec else bshape[1]
            if A.dim() != 2 or A.shape[1] != n or len(bshape) > 2 or bshape[0] != n:
                raise ValueError(f"system {i}: A must be (n, n) and B (n,) or (n, k)")
            S = arr[i]
            S.lda = _check_operand(A, f"A[{i}]", dev, adt, (n, n))
            ldb = _check_operand(B, f"B[{i}]", dev, vdt, bshape)
            X = outs[i] if outs is not None else torch.empty_like(B)
            ldx = _check_operand(X, f"out[{i}]", dev, vdt, bshape)
            if x0 is not None:
                if _check_operand(x0, f"x0[{i}]", dev, vdt, bshape) != ldx:
                    # X0 is read with X's leading dimension
                    x0 = torch.empty((n, ldx), dtype=vdt, device=dev)[:, :k].copy_(x0)
                S.X0 = x0.data_ptr()
            self._keep.append((A, B, x0))
            S.n = n
            S.k = k
            S.A = A.data_ptr()
            S.B = B.data_ptr()
            S.ldb = ldb
            S.X = X.data_ptr()
            S.ldx = ldx
            self.xs.append(X)

    def solve(self, *, stream=None, tol=1e-8, max_iter=10000, norm="inf"):
        """Solve every system once; returns (list of X, list of info dicts)."""
        from . import _stream_handle, make_options, status_string
        if self.count == 0:
            return [], []
        o = make_options(tol=tol, max_iter=max_iter, norm=norm)
        infos = (_lib.Info * self.count)()
        lib = self._lib
        st = lib.jacobi_solve_batched(self.ctx.handle if self.ctx else None, self.count,
                                      self._arr, self.dtype, ctypes.byref(o),
                                      _stream_handle(stream, self.device), infos)
        if st != 0:
            raise RuntimeError(f"jacobi_solve_batched: {status_string(st)}: "
                               f"{lib.jacobi_last_error().decode()}")
        out = []
        for i in range(self.count):
            d = infos[i].as_dict()
            d["status_name"] = status_string(d["status"])
            out.append(d)
        return self.xs, out


def solve_batched(systems, *, outs=None, ctx=None, stream=None, tol=1e-8, max_iter=10000,
                  norm="inf"):
    """Solve each (A, B) or (A, B, x0) in `systems` on the GPU.

    All A share one dtype: float32 or bfloat16 (B, x0 float32, k <= 32; one
    persistent MFMA launch), or float64 (systems solved one after another).
    Returns (list of X, list of info dicts)."""
    return Batch(systems, outs=outs, ctx=ctx).solve(stream=stream, tol=tol, max_iter=max_iter,
                                                    norm=norm)
